"""GPU parity of the adjoint gradient of the trajectory ensemble against the
FP64 oracle (reverse sweep of oracle.adjoint, pinned there by parameter shift).

E(theta) = sum_a w_a <psi_a|O|psi_a> with the ensemble weights of the
trajectory set (draw counts for multiplicity allocation, p_a for reweight).
The oracle takes its own PTS records and weights (oracle.pts.sample_kraus),
which must equal the library's.  Bar (complex64 states, FP64 reductions):
|E - E_ref| <= 1e-5, ||g - g_ref||_2 / ||g_ref||_2 <= 1e-4 and
max_i |g_i - g_ref_i| <= 1e-4 ||g_ref||_inf; complex128: 1e-10 throughout.
At the 16-qubit HEA size (1024 draws, 256 parameters) the whole set is
compared with oracle values stored by tests/golden/make_golden.py.
"""

import os

import numpy as np
import pytest
import torch

import paper_2504_16297_amd as P
from gpu_helpers import log
from oracle.adjoint import ensemble_value_and_grad
from oracle.noise import site_probs
from oracle.pts import ensemble_weights, sample_kraus
from workloads import c5_workload, random_small_circuit
from workloads.circuits import hea_circuit, zz_ring

pytestmark = pytest.mark.gpu

GOLDEN_C5 = os.path.join(os.path.dirname(__file__), "golden", "c5_ensemble_gradient.npz")


def _sample(plan, circ, pts, seed, cfg):
    """The library's trajectory set and the oracle's own PTS result (equal records)."""
    kw = {k: pts[k] for k in ("n_draws", "k_max", "total_shots") if k in pts}
    ts = P.ptsbe_sample_kraus(plan, pts["mode"], alloc=pts["alloc"], seed=seed, cfg=cfg, **kw)
    ref = sample_kraus(site_probs(circ), pts, seed, cfg)
    assert ts.get()["records"] == ref["records"]
    assert list(ts.weights()) == ref["weights"]
    return ts, ref


def _prop(n_draws):
    return {"mode": "proportional", "n_draws": n_draws, "total_shots": n_draws, "alloc": "multiplicity"}


def _gpu(plan, ts, params, obs, max_batch=0):
    E, G = P.ptsbe_adjoint_grad(plan, ts, params, obs, max_batch=max_batch)
    torch.cuda.synchronize()
    return float(E.cpu().numpy()[0]), G.cpu().numpy()


def _grad_errors(G, Gr):
    d = G - Gr
    return float(np.linalg.norm(d) / np.linalg.norm(Gr)), float(np.max(np.abs(d)) / np.max(np.abs(Gr)))


def _assert_close(E, G, Er, Gr, prec, what=""):
    rel2, relinf = _grad_errors(G, Gr)
    tol = 1e-4 if prec == "c64" else 1e-10
    log(f"  {what}E={E:.8f} ref={Er:.8f} |dE|={abs(E - Er):.2e} grad rel err l2={rel2:.2e} "
        f"max={relinf:.2e} ({G.size} params)")
    assert abs(E - Er) <= (1e-5 if prec == "c64" else 1e-10)
    assert rel2 <= tol and relinf <= tol


def _check(circ, plan, ts, recs, weights, params, obs, prec, max_batch=0):
    E, G = _gpu(plan, ts, params, obs, max_batch)
    Er, Gr = ensemble_value_and_grad(circ, recs, weights, params, obs)
    _assert_close(E, G, Er, Gr, prec)


@pytest.mark.parametrize("n,layers,prec,tile", [(4, 2, "c64", 0), (6, 3, "c128", 0), (8, 4, "c64", 5),
                                                (10, 3, "c64", 0), (10, 3, "c128", 6), (12, 2, "c64", 0)])
def test_hea_gradient(n, layers, prec, tile):
    log(f"[adjoint hea] n={n} layers={layers} {prec} tile={tile}")
    circ = hea_circuit(n, layers, np.random.default_rng(50 + n), 2e-2)
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ, precision=prec, tile_qubits=tile)
    ts, ref = _sample(plan, circ, _prop(40), 9, 5)
    _check(circ, plan, ts, ref["records"], ref["weights"], params, zz_ring(n), prec)


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
    ts, ref = _sample(plan, circ, _prop(24), 4, 7)
    _check(circ, plan, ts, ref["records"], ref["weights"], params, obs, prec)


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
    ts, ref = _sample(plan, circ, _prop(16), 2, 3)
    _check(circ, plan, ts, ref["records"], ref["weights"], params, [(1.0, (0, 1)), (0.5, (3,))], "c128")


def test_batches_split_by_workspace():
    """max_batch below the trajectory count: several psi/lambda batches, same result."""
    circ = hea_circuit(7, 3, np.random.default_rng(3), 3e-2)
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ, precision="c128")
    ts, ref = _sample(plan, circ, _prop(50), 1, 5)
    E1, G1 = _gpu(plan, ts, params, zz_ring(7))
    E2, G2 = _gpu(plan, ts, params, zz_ring(7), max_batch=3)
    assert abs(E1 - E2) <= 1e-12
    assert float(np.max(np.abs(G1 - G2))) <= 1e-12
    _check(circ, plan, ts, ref["records"], ref["weights"], params, zz_ring(7), "c128", max_batch=3)


def test_shared_prefix_matches_single_trajectories():
    """The forward preparation shares the error-free prefix across a set's
    trajectories; each trajectory alone (nothing to share) gives its own
    value and gradient, and their weighted sum equals the set's (complex128)."""
    circ = hea_circuit(9, 3, np.random.default_rng(12), 1e-2)
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ, precision="c128")
    ts, _ = _sample(plan, circ, _prop(40), 4, 6)
    B = ts.n_traj
    assert B >= 3
    E, G = _gpu(plan, ts, params, zz_ring(9))
    w = ts.weights()
    Es, Gs = 0.0, np.zeros_like(G)
    for a in range(B):
        Ea, Ga = _gpu(plan, ts.slice(a, a + 1), params, zz_ring(9))
        Es += w[a] * Ea
        Gs += w[a] * Ga
    assert abs(E - Es) <= 1e-12
    assert float(np.max(np.abs(G - Gs))) <= 1e-12


def test_deterministic_repeat():
    circ = hea_circuit(9, 3, np.random.default_rng(8), 2e-2)
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ)
    ts, _ = _sample(plan, circ, _prop(30), 6, 5)
    E1, G1 = _gpu(plan, ts, params, zz_ring(9))
    E2, G2 = _gpu(plan, ts, params, zz_ring(9))
    assert E1 == E2 and np.array_equal(G1, G2)


def test_hea16_full_size():
    """The 16-qubit, 8-layer HEA with 1024 proportional draws (256 parameters),
    run exactly as the gradient benchmark runs it: the whole set's E and
    gradient against the oracle's (stored by tests/golden/make_golden.py from
    the oracle's own records); the expectation mode's device-weighted E equals
    the adjoint call's; a 4-trajectory slice against the oracle directly."""
    wl = c5_workload()
    circ, obs = wl["circuit"], wl["observable"]
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ, precision=wl["precision"])
    ts, ref = _sample(plan, circ, wl["pts"], wl["seed"], wl["cfg"])
    log(f"[adjoint C5] trajectories={ts.n_traj}")
    gold = np.load(GOLDEN_C5)
    assert int(gold["n_traj"]) == ts.n_traj
    assert np.array_equal(gold["counts"], np.asarray(ref["counts"], dtype=np.float64))
    E, G = _gpu(plan, ts, params, obs)
    _assert_close(E, G, float(gold["E"]), gold["grad"], "c64", "whole set: ")
    r = P.ptsbe_run_batch(plan, ts, mode="expectation", params=params, observable=obs)
    torch.cuda.synchronize()
    Ee = float(r["E"].cpu()[0])
    Ew = float(np.dot(ts.weights(), r["expval"][:ts.n_traj].cpu().numpy()))
    log(f"  expectation mode E={Ee:.8f} (adjoint {E:.8f})")
    assert abs(Ee - E) <= 1e-6 and abs(Ee - Ew) <= 1e-12
    sub = ts.slice(0, 4)
    w = ensemble_weights(ref["counts"][:4], ref["p"][:4], "multiplicity")
    _check(circ, plan, sub, ref["records"][:4], w, params, obs, "c64")


def test_most_likely_set_uses_probability_weights():
    """A most-likely-first set (reweight allocation): E and gradient weight each
    trajectory by p_alpha / sum p (Sec. 3.1), as the oracle does."""
    circ = hea_circuit(8, 3, np.random.default_rng(41), 3e-2)
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ)
    pts = {"mode": "most_likely", "k_max": 40, "total_shots": 10 ** 5, "alloc": "reweight"}
    ts, ref = _sample(plan, circ, pts, 0, 5)
    w = np.asarray(ref["weights"])
    p = np.asarray(ref["p"])
    assert np.allclose(w, p / p.sum(), rtol=1e-13, atol=0)
    _check(circ, plan, ts, ref["records"], ref["weights"], params, zz_ring(8), "c64")


def test_autograd_function_and_central_differences():
    """torch.autograd through the adjoint call; complex128 central differences
    (h = 1e-4) of the GPU's own expectation agree to the FD error."""
    from paper_2504_16297_amd.autograd import expectation
    circ = hea_circuit(8, 3, np.random.default_rng(31), 2e-2)
    plan = P.ptsbe_plan(circ, precision="c128")
    ts, _ = _sample(plan, circ, _prop(30), 2, 5)
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
    ts, ref = _sample(plan, circ, _prop(24), 9, 5)
    obs = zz_ring(n)
    E, G = P.ptsbe_adjoint_grad(plan, ts, params, obs, max_batch=max_batch, seed=13, cfg=3)
    torch.cuda.synchronize()
    E, G = float(E.cpu().numpy()[0]), G.cpu().numpy()
    Er, Gr = ensemble_value_and_grad(circ, ref["records"], ref["weights"], params, obs, be_seed=(13, 3))
    _assert_close(E, G, Er, Gr, prec)


@pytest.mark.parametrize("n,prec,max_batch", [(6, "c64", 0), (7, "c128", 0), (14, "c64", 4)])
def test_gradient_through_dense_state_dependent_channels(n, prec, max_batch):
    """A 1-qubit channel with non-diagonal K^dagger K after every RY and a
    2-qubit joint decay after every ring CZ, each resolved from the reduced
    density matrix of its qubits in the forward preparation, checkpointed, and
    in the reverse sweep restored with (factor K_k)^dagger applied to lambda:
    E and the gradient equal the oracle's with the same decisions."""
    from test_gpu_parity import _dense_channels
    log(f"[adjoint dense state-dependent] n={n} {prec} max_batch={max_batch}")
    circ = hea_circuit(n, 2, np.random.default_rng(90 + n), 0.0)
    ch = _dense_channels()
    circ["channels"] = ch
    circ["rules"] = [{"when": "after_tag", "tag": "RY", "channel": 0}, {"when": "after_tag", "tag": "CZ", "channel": 1}]
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ, precision=prec)
    assert plan.info["n_sites"] == 0 and plan.info["n_measure"] >= 2 * n
    ts = P.ptsbe_trajset_from_records(plan, [()] * 6, [1] * 6)
    obs = zz_ring(n)
    E, G = P.ptsbe_adjoint_grad(plan, ts, params, obs, max_batch=max_batch, seed=13, cfg=3)
    torch.cuda.synchronize()
    E, G = float(E.cpu().numpy()[0]), G.cpu().numpy()
    Er, Gr = ensemble_value_and_grad(circ, [()] * 6, [1 / 6] * 6, params, obs, be_seed=(13, 3))
    _assert_close(E, G, Er, Gr, prec)
