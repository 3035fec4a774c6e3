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
