"""CPU check of the planner's fused device program: the exported tile passes,
slot matrices, overrides and measure-reset steps, run by a NumPy emulator,
reproduce the oracle's states and records."""

import numpy as np
import pytest

import paper_2504_16297_amd as P
from oracle.adjoint import ensemble_value_and_grad, observable_diag
from program_emulator import export_adjoint_tables, export_tables, run_adjoint, run_program
from oracle.noise import expand, site_channels
from oracle.statevector import run_record
from oracle.stabilizer import frame_run
from workloads import c1_workload, c3_workload, random_small_circuit
from workloads.circuits import hea_circuit, zz_ring


def _check(circ, plan, ts, params=None, tol=1e-10):
    g = ts.get()
    states, bits = run_program(export_tables(ts, params), circ["n_qubits"], len(g["m"]))
    ss = expand(circ)
    ch = site_channels(circ)
    for a, rec in enumerate(g["records"]):
        psi, b = run_record(circ, rec, params=params, steps_sites=ss, chans=ch)
        psi = psi / np.linalg.norm(psi)
        assert np.max(np.abs(states[a] - psi)) < tol, f"trajectory {a}"
        assert bits[a] == b


@pytest.mark.parametrize("n,tile,prec", [(1, 0, "c128"), (3, 0, "c128"), (5, 4, "c128"), (7, 4, "c128"),
                                         (8, 5, "c128"), (9, 6, "c128"), (10, 7, "c128"), (12, 6, "c128")])
def test_random_circuits_program(n, tile, prec):
    rng = np.random.default_rng(40 + n + tile)
    circ = random_small_circuit(n, 60, rng, p1=0.25, p2=0.3, with_params=True)
    plan = P.ptsbe_plan(circ, precision=prec, tile_qubits=tile)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=12, total_shots=12, seed=2, cfg=1)
    _check(circ, plan, ts, params=np.asarray(circ["params"]))


def test_c1_program():
    wl = c1_workload()
    plan = P.ptsbe_plan(wl["circuit"], precision="c128", tile_qubits=6)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=8, total_shots=8, seed=0, cfg=1)
    _check(wl["circuit"], plan, ts)


def test_hea_program_with_parameters():
    circ = hea_circuit(8, 3, np.random.default_rng(1), 0.1)
    plan = P.ptsbe_plan(circ, precision="c128", tile_qubits=5)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=10, total_shots=10, seed=0, cfg=5)
    _check(circ, plan, ts, params=np.asarray(circ["params"]))


def test_surface_code_program_records():
    """Measure-reset records of the fused program against Pauli frames (all of the
    first 120 most-likely records), and full states against the oracle for a few."""
    wl = c3_workload()
    circ = wl["circuit"]
    plan = P.ptsbe_plan(circ, precision="c128")
    ts = P.ptsbe_sample_kraus(plan, "most_likely", k_max=120, total_shots=120)
    g = ts.get()
    tabs = export_tables(ts)
    sub = list(range(0, 120, 7))
    ts_sub = P.ptsbe_trajset_from_records(plan, [g["records"][a] for a in sub], [1] * len(sub))
    states, bits = run_program(export_tables(ts_sub), 17, len(sub))
    for j, a in enumerate(sub):
        fb, _ = frame_run(circ, g["records"][a])
        assert bits[j] == fb, f"trajectory {a}: {g['records'][a]}"
    del tabs


@pytest.mark.parametrize("n,tile,prec", [(6, 0, "c128"), (8, 5, "c64"), (9, 6, "c128")])
def test_adjoint_program_gradient(n, tile, prec):
    """The reverse-sweep tables, run by the emulator, give the oracle's adjoint
    gradient (itself pinned by parameter shift)."""
    circ = random_small_circuit(n, 60, np.random.default_rng(40 + n), p1=0.1, p2=0.15, with_params=True)
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ, precision=prec, tile_qubits=tile)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=6, total_shots=6, seed=3, cfg=7)
    g = ts.get()
    w = g["count"].astype(np.float64) / g["count"].sum()
    obs = [(0.7, (0,)), (-1.3, (1, n - 1)), (0.4, tuple(range(n)))]
    fwd = export_tables(ts, params)
    adj, dot_param = export_adjoint_tables(ts, params)
    tol = 1e-5 if prec == "c64" else 1e-10
    E, G = run_adjoint(fwd, adj, dot_param, n, ts.n_traj, params.size, observable_diag(n, obs), w,
                       back_tol=1e-9 if prec == "c128" else 1e-5)
    Er, Gr = ensemble_value_and_grad(circ, g["records"], w, params, obs)
    assert abs(E - Er) <= tol
    assert np.max(np.abs(G - Gr)) <= tol * max(1.0, np.max(np.abs(Gr)))


def test_adjoint_program_hea():
    circ = hea_circuit(7, 3, np.random.default_rng(5), 0.03)
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ, precision="c128")
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=5, total_shots=5, seed=1, cfg=5)
    g = ts.get()
    w = g["count"].astype(np.float64) / g["count"].sum()
    fwd = export_tables(ts, params)
    adj, dot_param = export_adjoint_tables(ts, params)
    assert sorted(set(dot_param.tolist())) == list(range(params.size))
    E, G = run_adjoint(fwd, adj, dot_param, 7, ts.n_traj, params.size, observable_diag(7, zz_ring(7)), w)
    Er, Gr = ensemble_value_and_grad(circ, g["records"], w, params, zz_ring(7))
    assert abs(E - Er) <= 1e-10
    assert np.max(np.abs(G - Gr)) <= 1e-10 * max(1.0, np.max(np.abs(Gr)))


def _slot_diag_imag(t):
    """Largest |Im| of the diagonal of each 2x2 default slot matrix, per pass."""
    out = []
    for ps in t["passes"]:
        ops = t["ops"][ps["op_begin"]:ps["op_begin"] + ps["n_ops"]]
        for op in ops:
            ty = int(op["type"])
            js = [j for j in range(4) if (int(op["mask"]) >> j) & 1] if ty == 8 else ([0] if ty == 1 else [])
            for j in js:
                off = int(t["slot_default"][int(ps["slot_begin"]) + int(op["slots"][j])])
                m = t["pool"][off:off + 4]
                out.append(max(abs(m[0].imag), abs(m[3].imag)))
    return np.asarray(out)


def test_phase_frames_keep_states_and_make_real_diagonals():
    """Phase frames (Sec. 3's trajectories are fixed circuits, so a diagonal
    can be carried between two matrices of a qubit): the rewritten tables give
    the same states as the plain ones and as the oracle, for trajectories with
    overrides on rewritten slots, and most 2x2 slots of a brick circuit (every
    U3 followed by another matrix on its qubit) end up with a real diagonal."""
    from workloads.circuits import brick_circuit
    import math
    circ = brick_circuit(8, 6, np.random.default_rng(5), 0.05, 0.08, eps_sigma=0.02)
    framed = P.ptsbe_plan(circ, precision="c128", tile_qubits=6, pair_fusion=False)
    plain = P.ptsbe_plan(circ, precision="c128", tile_qubits=6, phase_frames=False, pair_fusion=False)
    ts_f = P.ptsbe_sample_kraus(framed, "proportional", n_draws=16, total_shots=16, seed=4, cfg=2)
    ts_p = P.ptsbe_sample_kraus(plain, "proportional", n_draws=16, total_shots=16, seed=4, cfg=2)
    tf, tp = export_tables(ts_f), export_tables(ts_p)
    imf, imp = _slot_diag_imag(tf), _slot_diag_imag(tp)
    assert len(imf) == len(imp)
    # 8 qubits x 6 layers of U3: all but the last matrix of each qubit are rewritten
    assert np.sum(imf < 1e-12) >= 8 * 5
    assert np.sum(imp < 1e-12) < np.sum(imf < 1e-12)
    g = ts_f.get()
    assert any(len(r) for r in g["records"])
    sf, _ = run_program(tf, 8, len(g["m"]))
    sp, _ = run_program(tp, 8, len(g["m"]))
    assert max(float(np.max(np.abs(a - b))) for a, b in zip(sf, sp)) < 1e-12
    _check(circ, framed, ts_f)


def test_phase_frames_absorb_diagonals_and_flush_before_measure_reset():
    """A diagonal gate between two matrices of its qubit is merged away (its
    slot holds the identity), and no diagonal stays pending across a
    measure-reset: the surface-code program (measure-resets between rounds)
    still matches the oracle record by record."""
    circ = {"n_qubits": 3, "channels": [{"name": "depolarizing", "nq": 1, "p": 0.2}], "rules": [],
            "params": [], "ops": [
                {"kind": "gate", "name": "H", "qubits": (0,), "params": ()},
                {"kind": "gate", "name": "CNOT", "qubits": (0, 1), "params": ()},
                {"kind": "gate", "name": "RZ", "qubits": (2,), "params": (0.3,)},
                {"kind": "gate", "name": "CZ", "qubits": (1, 2), "params": ()},
                {"kind": "gate", "name": "RZ", "qubits": (2,), "params": (0.7,)},
                {"kind": "gate", "name": "CZ", "qubits": (0, 2), "params": ()},
                {"kind": "gate", "name": "H", "qubits": (2,), "params": ()},
                {"kind": "noise", "channel": 0, "qubits": (2,)},
                {"kind": "gate", "name": "U3", "qubits": (1,), "params": (0.4, 0.1, 0.9)},
                {"kind": "gate", "name": "RX", "qubits": (2,), "params": (0.5,)},
            ]}
    plan = P.ptsbe_plan(circ, precision="c128")
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=8, total_shots=8, seed=1, cfg=1)
    _check(circ, plan, ts)

    def identity_slots(t):
        ops = t["ops"]
        n_id = 0
        for op in ops:
            if int(op["type"]) != 1:
                continue
            off = int(t["slot_default"][int(op["slots"][0])])
            n_id += int(np.allclose(t["pool"][off:off + 4], [1, 0, 0, 1], atol=1e-15))
        return n_id
    plain = P.ptsbe_plan(circ, precision="c128", phase_frames=False)
    ts_p = P.ptsbe_sample_kraus(plain, "proportional", n_draws=8, total_shots=8, seed=1, cfg=1)
    # the two RZ slots on qubit 2 sit between matrices of that qubit
    assert identity_slots(export_tables(ts)) == identity_slots(export_tables(ts_p)) + 2
    wl = c3_workload(rounds=1)
    plan3 = P.ptsbe_plan(wl["circuit"], precision="c128")
    ts3 = P.ptsbe_sample_kraus(plan3, "most_likely", k_max=12, total_shots=12, seed=0, cfg=3)
    _check(wl["circuit"], plan3, ts3)
