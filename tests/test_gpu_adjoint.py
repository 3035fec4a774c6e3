"""GPU parity of the adjoint gradient of the trajectory ensemble against the
FP64 oracle (reverse sweep of oracle.adjoint, pinned there by parameter shift).

E(theta) = sum_a w_a <psi_a|O|psi_a>, w_a = count_a / sum count.  Bar: E within
1e-5 absolute and every gradient entry within 1e-4 of max|grad| for complex64
states (1e-10 for complex128).  At the 16-qubit HEA size (1024 draws) the
oracle checks a slice of trajectories one by one, and the full set is checked
against the GPU's own parameter-shift differences of its expectation mode, a
property that holds at any size.
"""

import numpy as np
import pytest
import torch

import paper_2504_16297_amd as P
from gpu_helpers import log
from oracle.adjoint import ensemble_value_and_grad
from workloads import c5_workload, random_small_circuit
from workloads.circuits import hea_circuit, zz_ring

pytestmark = pytest.mark.gpu


def _weights(g):
    c = g["count"].astype(np.float64)
    return c / c.sum()


def _gpu(plan, ts, params, obs, max_batch=0):
    E, G = P.ptsbe_adjoint_grad(plan, ts, params, obs, max_batch=max_batch)
    torch.cuda.synchronize()
    return float(E.cpu().numpy()[0]), G.cpu().numpy()


def _check(circ, plan, ts, params, obs, prec, max_batch=0):
    g = ts.get()
    E, G = _gpu(plan, ts, params, obs, max_batch)
    Er, Gr = ensemble_value_and_grad(circ, g["records"], _weights(g), params, obs)
    scale = max(1.0, float(np.max(np.abs(Gr))))
    tol = 1e-4 if prec == "c64" else 1e-10
    err = float(np.max(np.abs(G - Gr))) / scale
    log(f"  E={E:.6f} ref={Er:.6f} |dE|={abs(E - Er):.2e} grad rel err={err:.2e} ({len(params)} params)")
    assert abs(E - Er) <= (1e-5 if prec == "c64" else 1e-10)
    assert err <= tol


@pytest.mark.parametrize("n,layers,prec,tile", [(4, 2, "c64", 0), (6, 3, "c128", 0), (8, 4, "c64", 5),
                                                (10, 3, "c64", 0), (10, 3, "c128", 6), (12, 2, "c64", 0)])
def test_hea_gradient(n, layers, prec, tile):
    log(f"[adjoint hea] n={n} layers={layers} {prec} tile={tile}")
    circ = hea_circuit(n, layers, np.random.default_rng(50 + n), 2e-2)
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ, precision=prec, tile_qubits=tile)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=40, total_shots=40, seed=9, cfg=5)
    _check(circ, plan, ts, params, zz_ring(n), prec)


@pytest.mark.parametrize("n,gates,prec,tile", [(5, 40, "c64", 0), (7, 60, "c128", 0), (9, 80, "c64", 5),
                                               (11, 70, "c64", 0)])
def test_random_circuit_gradient(n, gates, prec, tile):
    """X, Y and Z generators, 2-qubit gates on arbitrary pairs, Pauli and U3-mixture noise."""
    log(f"[adjoint random] n={n} gates={gates} {prec} tile={tile}")
    rng = np.random.default_rng(300 + n)
    circ = random_small_circuit(n, gates, rng, p1=0.1, p2=0.15, with_params=True)
    params = np.asarray(circ["params"])
    assert params.size > 0
    obs = [(0.7, (0,)), (-1.3, (1, n - 1)), (0.4, tuple(range(n)))]
    plan = P.ptsbe_plan(circ, precision=prec, tile_qubits=tile)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=24, total_shots=24, seed=4, cfg=7)
    _check(circ, plan, ts, params, obs, prec)


def test_shared_parameters_accumulate():
    """A parameter used by several gates receives the sum of their contributions."""
    rng = np.random.default_rng(12)
    circ = random_small_circuit(6, 60, rng, with_params=True)
    k = 0
    for op in circ["ops"]:
        if op["kind"] == "param":
            op["index"] = k % 3
            k += 1
    circ["params"] = circ["params"][:3]
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ, precision="c128")
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=16, total_shots=16, seed=2, cfg=3)
    _check(circ, plan, ts, params, [(1.0, (0, 1)), (0.5, (3,))], "c128")


def test_batches_split_by_workspace():
    """max_batch below the trajectory count: several psi/lambda batches, same result."""
    circ = hea_circuit(7, 3, np.random.default_rng(3), 3e-2)
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ, precision="c128")
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=50, total_shots=50, seed=1, cfg=5)
    E1, G1 = _gpu(plan, ts, params, zz_ring(7))
    E2, G2 = _gpu(plan, ts, params, zz_ring(7), max_batch=3)
    assert abs(E1 - E2) <= 1e-12
    assert float(np.max(np.abs(G1 - G2))) <= 1e-12
    _check(circ, plan, ts, params, zz_ring(7), "c128", max_batch=3)


def test_deterministic_repeat():
    circ = hea_circuit(9, 3, np.random.default_rng(8), 2e-2)
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=30, total_shots=30, seed=6, cfg=5)
    E1, G1 = _gpu(plan, ts, params, zz_ring(9))
    E2, G2 = _gpu(plan, ts, params, zz_ring(9))
    assert E1 == E2 and np.array_equal(G1, G2)


def test_hea16_full_size():
    """The 16-qubit, 8-layer HEA with 1024 proportional draws (256 parameters):
    a slice of trajectories against the oracle, the whole set against the GPU's
    own parameter-shift differences on sampled parameters."""
    wl = c5_workload()
    circ, obs = wl["circuit"], wl["observable"]
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ, precision=wl["precision"])
    pts = wl["pts"]
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=pts["n_draws"], total_shots=pts["total_shots"],
                              seed=wl["seed"], cfg=wl["cfg"])
    log(f"[adjoint C5] trajectories={ts.n_traj}")
    sub = ts.slice(0, 4)
    _check(circ, plan, sub, params, obs, "c64")
    E, G = _gpu(plan, ts, params, obs)
    g = ts.get()
    w = _weights(g)

    def expect(pv):
        r = P.ptsbe_run_batch(plan, ts, mode="expectation", params=pv, observable=obs)
        torch.cuda.synchronize()
        return float(np.dot(w, r["expval"].cpu().numpy()))

    assert abs(expect(params) - E) <= 1e-6
    rng = np.random.default_rng(0)
    for i in rng.choice(params.size, size=6, replace=False):
        pp = params.copy(); pp[i] += np.pi / 2
        pm = params.copy(); pm[i] -= np.pi / 2
        shift = 0.5 * (expect(pp) - expect(pm))
        log(f"  param {i}: adjoint {G[i]:+.6f} shift {shift:+.6f}")
        assert abs(G[i] - shift) <= 1e-4 * max(1.0, float(np.max(np.abs(G))))


def test_autograd_function_and_central_differences():
    """torch.autograd through the adjoint call; complex128 central differences
    (h = 1e-4) of the GPU's own expectation agree to the FD error."""
    from paper_2504_16297_amd.autograd import expectation
    circ = hea_circuit(8, 3, np.random.default_rng(31), 2e-2)
    plan = P.ptsbe_plan(circ, precision="c128")
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=30, total_shots=30, seed=2, cfg=5)
    obs = zz_ring(8)
    th = torch.tensor(circ["params"], dtype=torch.float64, device="cuda", requires_grad=True)
    E = expectation(th, plan, ts, obs)
    E.backward()
    g = th.grad.cpu().numpy()
    E2, G2 = _gpu(plan, ts, np.asarray(circ["params"]), obs)
    assert abs(float(E) - E2) <= 1e-12 and np.array_equal(g, G2)
    h = 1e-4
    base = np.asarray(circ["params"])
    fd = np.zeros(base.size)
    with torch.no_grad():
        for i in range(base.size):
            pp = base.copy(); pp[i] += h
            pm = base.copy(); pm[i] -= h
            ep = float(expectation(torch.tensor(pp, device="cuda"), plan, ts, obs))
            em = float(expectation(torch.tensor(pm, device="cuda"), plan, ts, obs))
            fd[i] = (ep - em) / (2 * h)
    err = float(np.max(np.abs(fd - g)))
    log(f"  autograd vs central FD (c128, h=1e-4): max|d| = {err:.2e}")
    assert err <= 1e-6


@pytest.mark.parametrize("n,prec,tile,max_batch", [(5, "c64", 0, 0), (7, "c128", 0, 0), (9, "c64", 5, 0),
                                                   (8, "c64", 0, 5)])
def test_gradient_through_state_dependent_channels(n, prec, tile, max_batch):
    """Amplitude damping after every RY, decided on the device as a batched run
    decides it (key (seed, cfg, trajectory)), the state at each decision
    checkpointed and restored by the reverse sweep with the chosen operator
    held fixed; depolarizing after every CZ from the trajectory records.  E and
    the gradient equal the oracle's (same decisions, same fixed operators)."""
    log(f"[adjoint state-dependent] n={n} {prec} tile={tile} max_batch={max_batch}")
    circ = hea_circuit(n, 2, np.random.default_rng(70 + n), 2e-2)
    circ["channels"].append({"name": "amplitude_damping", "gamma": 0.2, "nq": 1})
    circ["rules"].append({"when": "after_tag", "tag": "RY", "channel": 1})
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ, precision=prec, tile_qubits=tile)
    assert plan.info["n_measure"] == 2 * n
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=24, total_shots=24, seed=9, cfg=5)
    g = ts.get()
    obs = zz_ring(n)
    E, G = P.ptsbe_adjoint_grad(plan, ts, params, obs, max_batch=max_batch, seed=13, cfg=3)
    torch.cuda.synchronize()
    E, G = float(E.cpu().numpy()[0]), G.cpu().numpy()
    Er, Gr = ensemble_value_and_grad(circ, g["records"], _weights(g), params, obs, be_seed=(13, 3))
    scale = max(1.0, float(np.max(np.abs(Gr))))
    err = float(np.max(np.abs(G - Gr))) / scale
    log(f"  E={E:.6f} ref={Er:.6f} |dE|={abs(E - Er):.2e} grad rel err={err:.2e}")
    assert abs(E - Er) <= (1e-5 if prec == "c64" else 1e-10)
    assert err <= (1e-4 if prec == "c64" else 1e-10)
