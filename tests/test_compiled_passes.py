"""CPU check of the pass compiler: every generated pass kernel is compiled with
g++ against a thread-per-lane shim and run over the exported device tables
(tests/compiled_cpu.py); the states must equal the oracle's.  Covers register
changes, 2x2 groups, 4x4 matrices in registers and through the LDS tile,
diagonals on register, thread and tile bits, CZ-type signs on every kind of
bit, block-uniform phases, and measure-resets."""

import numpy as np
import pytest

import paper_2504_16297_amd as P
from paper_2504_16297_amd import _lib as L
from compiled_cpu import pass_source, run_compiled
from gpu_helpers import oracle_states
from workloads import c1_workload, c3_workload, random_small_circuit
from workloads.circuits import hea_circuit

CASES = [(6, 30, "c128", 0, 1), (8, 60, "c64", 0, 2), (10, 80, "c64", 0, 1070), (9, 70, "c128", 7, 5),
         (12, 70, "c64", 8, 9), (13, 60, "c128", 9, 13)]


RUNS = [c + (False,) for c in CASES] + [CASES[i] + (True,) for i in (1, 3, 4)]


@pytest.mark.parametrize("n,gates,prec,tile,seed,half", RUNS)
def test_random_circuits(n, gates, prec, tile, seed, half):
    circ = random_small_circuit(n, gates, np.random.default_rng(seed), p1=0.2, p2=0.3, with_params=True)
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ, precision=prec, tile_qubits=tile, half_tile=half)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=3, total_shots=3, seed=3, cfg=1)
    st = run_compiled(plan, ts, params)
    ref, _ = oracle_states(circ, ts.get()["records"], params=params)
    tol = 1e-5 if prec == "c64" else 1e-12
    assert max(float(np.max(np.abs(st[a] - ref[a]))) for a in range(len(ref))) <= tol


@pytest.mark.parametrize("half", [False, True])
def test_c1_slice(half):
    wl = c1_workload()
    plan = P.ptsbe_plan(wl["circuit"], precision="c128", half_tile=half)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=64, total_shots=64000, seed=0, cfg=1).slice(0, 4)
    st = run_compiled(plan, ts)
    ref, _ = oracle_states(wl["circuit"], ts.get()["records"])
    assert max(float(np.max(np.abs(st[a] - ref[a]))) for a in range(len(ref))) <= 1e-12


def test_surface_code_measure_resets():
    wl = c3_workload()
    plan = P.ptsbe_plan(wl["circuit"], precision="c64")
    ts = P.ptsbe_sample_kraus(plan, "most_likely", k_max=6, total_shots=60, seed=0, cfg=3).slice(0, 3)
    st = run_compiled(plan, ts)
    ref, _ = oracle_states(wl["circuit"], ts.get()["records"])
    assert max(float(np.max(np.abs(st[a] - ref[a]))) for a in range(len(ref))) <= 1e-5


def test_hea_with_parameters():
    circ = hea_circuit(8, 3, np.random.default_rng(4), 0.05)
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ, precision="c64")
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=4, total_shots=4, seed=1, cfg=5)
    st = run_compiled(plan, ts, params)
    ref, _ = oracle_states(circ, ts.get()["records"], params=params)
    assert max(float(np.max(np.abs(st[a] - ref[a]))) for a in range(len(ref))) <= 1e-5


def test_brick_half_tile_transposes():
    """A 14-qubit brick circuit with coherent over-rotations on 4096-amplitude
    tiles, register changes through half the tile: every pass is split."""
    from compiled_cpu import pass_source
    from workloads import brick_circuit
    circ = brick_circuit(14, 6, np.random.default_rng(3), 0.05, 0.08, eps_sigma=0.05)
    plan = P.ptsbe_plan(circ, half_tile=True)
    srcs = [pass_source(plan, p) for p in range(plan.info["n_passes"])]
    # every register change goes through half the tile (a 2048-amplitude window)
    assert any("tile[" in s for s in srcs)
    assert all("const uint32_t Lc = " in s for s in srcs if "tile[" in s)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=3, total_shots=3, seed=5, cfg=2)
    st = run_compiled(plan, ts)
    ref, _ = oracle_states(circ, ts.get()["records"])
    assert max(float(np.max(np.abs(st[a] - ref[a]))) for a in range(len(ref))) <= 1e-5


@pytest.mark.parametrize("n,prec,seed", [(7, "c128", 11), (9, "c64", 12)])
def test_adjoint_sweep_kernels(n, prec, seed):
    """The compiled reverse sweep (psi and lambda in registers, gradient terms
    as per-wavefront FP64 partials) against the oracle's adjoint gradient, on
    circuits with X, Y and Z generators, 2-qubit gates and noise."""
    from compiled_cpu import run_compiled_adjoint
    from oracle.adjoint import ensemble_value_and_grad, observable_diag
    circ = random_small_circuit(n, 50, np.random.default_rng(seed), p1=0.1, p2=0.15, with_params=True)
    params = np.asarray(circ["params"])
    obs = [(0.7, (0,)), (-1.3, (1, n - 1)), (0.4, tuple(range(n)))]
    plan = P.ptsbe_plan(circ, precision=prec)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=3, total_shots=3, seed=3, cfg=7)
    E, G = run_compiled_adjoint(plan, ts, params, observable_diag(n, obs))
    g = ts.get()
    w = g["count"].astype(np.float64) / g["count"].sum()
    Er, Gr = ensemble_value_and_grad(circ, g["records"], w, params, obs)
    tol = 1e-5 if prec == "c64" else 1e-11
    assert abs(E - Er) <= tol
    assert float(np.max(np.abs(G - Gr))) <= tol * max(1.0, float(np.max(np.abs(Gr))))


def test_adjoint_sweep_real_and_diagonal_forms():
    """Reverse sweep of a hardware-efficient ansatz: Y rotations that no record
    changes run as real 2x2 matrices, Z rotations as diagonals, noise slots
    (which records change) in the general form and only where the block's
    trajectory overrides them; the gradient equals the oracle's."""
    from compiled_cpu import pass_source, run_compiled_adjoint
    from oracle.adjoint import ensemble_value_and_grad, observable_diag
    from workloads.circuits import hea_circuit, zz_ring
    n = 8
    circ = hea_circuit(n, 3, np.random.default_rng(41), 0.2)
    params = np.asarray(circ["params"])
    plan = P.ptsbe_plan(circ)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=4, total_shots=4, seed=2, cfg=9)
    srcs = []  # every reverse-sweep pass (their count is not in the plan info)
    p = 0
    while True:
        try:
            srcs.append(pass_source(plan, p, adjoint=True))
        except P.PtsbeError:
            break
        p += 1
    body = "".join(srcs)
    assert "= crr(m0.x, x0, m1.x, x1)" in body     # real form
    assert "= cm(m0, s" in body and "= cm(m3, l" in body  # diagonal form, psi and lambda
    assert "= cf(m0, x0, m1, x1)" in body          # general form (noise slots)
    assert "  if (__builtin_expect((ovw" in body    # ... applied only where overridden
    assert "  } else {\n    s" in body               # CZ slots: negations unless overridden
    assert all("amdgpu_waves_per_eu(3)" in s for s in srcs if s)  # three waves per SIMD
    obs = zz_ring(n)
    E, G = run_compiled_adjoint(plan, ts, params, observable_diag(n, obs))
    g = ts.get()
    w = g["count"].astype(np.float64) / g["count"].sum()
    Er, Gr = ensemble_value_and_grad(circ, g["records"], w, params, obs)
    assert abs(E - Er) <= 1e-5
    assert float(np.max(np.abs(G - Gr))) <= 1e-5 * max(1.0, float(np.max(np.abs(Gr))))


@pytest.mark.parametrize("frames", [True, False])
def test_brick_phase_frames(frames):
    """Compiled passes of a brick circuit in phase frames: the fixed 2x2 slots
    run in the unit-diagonal form (x_r + c x_o, the diagonal with its magnitude
    pending) unless the block's trajectory overrides them (noise strong enough
    that most trajectories carry overrides), and the plain plan (no frames)
    keeps the general form; both match the oracle."""
    from compiled_cpu import pass_source
    from workloads import brick_circuit
    circ = brick_circuit(12, 5, np.random.default_rng(8), 0.08, 0.1, eps_sigma=0.05)
    plan = P.ptsbe_plan(circ, phase_frames=frames, pair_fusion=False)
    srcs = "".join(pass_source(plan, p) for p in range(plan.info["n_passes"]))
    assert ("= cu(x0, m1, x1)" in srcs) == frames      # fixed U3s: unit-diagonal rows
    assert ("  if (__builtin_expect((ovw" in srcs) == frames   # override branch of a rewritten slot
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=6, total_shots=6, seed=6, cfg=2)
    g = ts.get()
    assert sum(1 for r in g["records"] if len(r)) >= 2
    st = run_compiled(plan, ts)
    ref, _ = oracle_states(circ, g["records"])
    assert max(float(np.max(np.abs(st[a] - ref[a]))) for a in range(len(ref))) <= 1e-5


def test_brick_pair_fusion():
    """Pair fusion on a brick circuit: each even-layer CZ merges with the 2x2
    runs on its qubits into a 4x4 slot that also takes the next layer's gates on
    them, applied in registers (both bits register bits, no pass through the
    LDS tile for it), rows 0..2 in the unit-diagonal form of the phase frame;
    noise overrides of the 4x4 slots included, the states match the oracle, and
    the plan has fewer 2x2 register groups than without."""
    from collections import Counter
    from compiled_cpu import pass_source
    from paper_2504_16297_amd.tables import export_tables
    from workloads import brick_circuit
    circ = brick_circuit(12, 6, np.random.default_rng(9), 0.06, 0.1, eps_sigma=0.05)
    plan = P.ptsbe_plan(circ)
    srcs = [pass_source(plan, p) for p in range(plan.info["n_passes"])]
    assert any("cd4(M + " in s for s in srcs)                 # 4x4 in registers
    assert any("= cu3(x0, M[1], x1" in s for s in srcs)       # fixed 4x4s: rows 0..2 with a unit diagonal
    assert not any("cd4(m, x0" in s for s in srcs)            # never through the tile
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=6, total_shots=6, seed=7, cfg=2)
    g = ts.get()
    assert sum(1 for r in g["records"] if len(r)) >= 3
    ops = Counter(int(o["type"]) for o in export_tables(ts, None)["ops"])
    plain = P.ptsbe_plan(circ, pair_fusion=False)
    ts0 = P.ptsbe_sample_kraus(plain, "proportional", n_draws=6, total_shots=6, seed=7, cfg=2)
    ops0 = Counter(int(o["type"]) for o in export_tables(ts0, None)["ops"])
    assert ops[2] > 0 and ops0[2] == 0 and ops[8] < ops0[8]   # M2 slots, fewer M1G groups
    st = run_compiled(plan, ts)
    ref, _ = oracle_states(circ, g["records"])
    assert max(float(np.max(np.abs(st[a] - ref[a]))) for a in range(len(ref))) <= 1e-5


@pytest.mark.parametrize("tile", [0, 6])
def test_state_dependent_channels(tile):
    """Amplitude damping resolved when the state reaches it: the generated
    kernels apply K_k / sqrt(p_k) from the record entry, the decisions made
    between passes as the device makes them; states and entries equal the
    oracle's for every trajectory (alpha = its index)."""
    rng = np.random.default_rng(4)
    circ = random_small_circuit(8, 40, rng, p1=0.0, p2=0.0)
    circ = dict(circ, ops=[op for op in circ["ops"] if op["kind"] != "noise"],
                channels=[{"name": "amplitude_damping", "gamma": 0.25, "nq": 1},
                          {"name": "depolarizing", "nq": 1, "p": 0.05}],
                rules=[{"when": "after_tag", "tag": "U3", "channel": 0}, {"when": "after_tag", "tag": "RX", "channel": 1}])
    plan = P.ptsbe_plan(circ, tile_qubits=tile)
    assert any(c >= 0 for c, _ in plan.record_info())
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=6, total_shots=6, seed=3, cfg=1)
    st = run_compiled(plan, ts, circuit=circ, be=(9, 2))
    from oracle.statevector import run_record
    for a, rec in enumerate(ts.get()["records"]):
        psi, entries = run_record(circ, rec, be_key=(9, 2, a))
        psi = psi / np.linalg.norm(psi)
        assert float(np.max(np.abs(st[a] - psi))) <= 1e-5, f"trajectory {a}"


@pytest.mark.parametrize("swizzle,nontemporal", [(True, False), (False, False), (True, True), (None, False)])
def test_swizzled_state_storage(swizzle, nontemporal):
    """States above 2^12 amplitudes stored swizzled (runs of 16 amplitudes and
    blocks of 4096 kept, high index bits XORed onto bits 4..11; forced here with
    PTSBE_PLAN_SWIZZLE, by default only from PTSBE_SWIZZLE_MIN_QUBITS qubits): the
    generated kernels address them that way, or plainly, and the states read
    back in index order equal the oracle's either way."""
    from compiled_cpu import storage_positions
    from workloads import brick_circuit
    pos = storage_positions(16)
    assert np.array_equal(np.sort(pos), np.arange(1 << 16))          # a permutation
    assert np.array_equal(pos[pos], np.arange(1 << 16))              # an involution
    assert np.array_equal(pos & 15, np.arange(1 << 16) & 15)         # 16-amplitude runs kept
    assert np.array_equal(pos >> 12, np.arange(1 << 16) >> 12)       # 4096-amplitude blocks kept
    circ = brick_circuit(15, 4, np.random.default_rng(6), 0.05, 0.1)
    plan = P.ptsbe_plan(circ, swizzle=swizzle, nontemporal=nontemporal)
    swizzle = bool(swizzle)                   # 15 qubits: plain order by default
    assert plan.info["swizzled"] == swizzle
    big = brick_circuit(L.SWIZZLE_MIN_QUBITS, 1, np.random.default_rng(1), 0.0, 0.0)
    assert P.ptsbe_plan(big).info["swizzled"] == 1
    below = brick_circuit(L.SWIZZLE_MIN_QUBITS - 1, 1, np.random.default_rng(1), 0.0, 0.0)
    assert P.ptsbe_plan(below).info["swizzled"] == 0
    src = "".join(pass_source(plan, p) for p in range(plan.info["n_passes"]))
    assert ("const uint64_t px = " in src) == swizzle
    assert ("stnt(dstp" in src) == nontemporal
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=3, total_shots=3, seed=2, cfg=2)
    st = run_compiled(plan, ts, swizzled=swizzle)
    ref, _ = oracle_states(circ, ts.get()["records"])
    assert max(float(np.max(np.abs(st[a] - ref[a]))) for a in range(len(ref))) <= 1e-5


@pytest.mark.parametrize("n,swizzle", [(14, True), (13, False), (17, True)])
def test_two_tiles_per_workgroup(n, swizzle):
    """PTSBE_PLAN_TWO_TILES: every forward pass kernel runs tiles 2b and 2b + 1
    of its state in workgroup b (the second tile's loads issued first, the
    registers swapped after the first tile's stores), including the
    initialising pass and, at 17 qubits (the surface code), passes with
    measure-resets; the states equal the oracle's and those of one tile per
    workgroup."""
    if n == 17:
        circ = c3_workload()["circuit"]
    else:
        from workloads import brick_circuit
        circ = brick_circuit(n, 4, np.random.default_rng(n), 0.05, 0.1)
    plan2 = P.ptsbe_plan(circ, swizzle=swizzle, two_tiles=True)
    plan1 = P.ptsbe_plan(circ, swizzle=swizzle)
    srcs = [pass_source(plan2, p) for p in range(plan2.info["n_passes"])]
    assert all("tile_id0 = 2ull * blockIdx.x" in s for s in srcs)
    assert any("s0.x = (base == 0 && tid == 0)" in s for s in srcs)      # the initialising pass
    if n == 17:
        assert plan2.info["n_measure"] > 0
        ts = P.ptsbe_sample_kraus(plan2, "most_likely", k_max=6, total_shots=60, seed=0, cfg=3).slice(0, 3)
    else:
        ts = P.ptsbe_sample_kraus(plan2, "proportional", n_draws=3, total_shots=3, seed=4, cfg=1)
    st2 = run_compiled(plan2, ts)
    st1 = run_compiled(plan1, ts)
    assert np.array_equal(st1, st2)
    ref, _ = oracle_states(circ, ts.get()["records"])
    assert max(float(np.max(np.abs(st2[a] - ref[a]))) for a in range(len(ref))) <= 1e-5


@pytest.mark.parametrize("n,swizzle,half", [(14, True, False), (13, None, False), (15, False, True)])
def test_thirteen_qubit_tiles(n, swizzle, half):
    """13-qubit tiles (512 threads x 16 amplitudes, 64 KiB of LDS, or 32 KiB in
    two rounds): fewer passes for the same circuit, the states equal the
    oracle's."""
    from workloads import brick_circuit
    circ = brick_circuit(n, 5, np.random.default_rng(40 + n), 0.05, 0.1, eps_sigma=0.05)
    plan = P.ptsbe_plan(circ, tile_qubits=13, swizzle=swizzle, half_tile=half)
    assert plan.info["tile_qubits"] == 13
    assert plan.info["n_passes"] <= P.ptsbe_plan(circ, tile_qubits=12).info["n_passes"]
    srcs = [pass_source(plan, p) for p in range(plan.info["n_passes"])]
    assert all("__launch_bounds__(512)" in s for s in srcs)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=3, total_shots=3, seed=6, cfg=2)
    st = run_compiled(plan, ts)
    ref, _ = oracle_states(circ, ts.get()["records"])
    assert max(float(np.max(np.abs(st[a] - ref[a]))) for a in range(len(ref))) <= 1e-5


def test_tile_search_windows():
    """The scheduler's tile search (the best of the greedy tile and windows of
    consecutive qubits) needs fewer passes on a brick circuit than the greedy
    tile alone, and its passes give the oracle's states."""
    from workloads import brick_circuit
    circ = brick_circuit(14, 12, np.random.default_rng(9), 0.05, 0.1)
    found = P.ptsbe_plan(circ, tile_qubits=8)
    greedy = P.ptsbe_plan(circ, tile_qubits=8, tile_search=False)
    assert found.info["n_passes"] < greedy.info["n_passes"]
    ts = P.ptsbe_sample_kraus(found, "proportional", n_draws=3, total_shots=3, seed=7, cfg=2)
    st = run_compiled(found, ts)
    ref, _ = oracle_states(circ, ts.get()["records"])
    assert max(float(np.max(np.abs(st[a] - ref[a]))) for a in range(len(ref))) <= 1e-5


def test_unit_and_real_diagonal_frames():
    """Slots whose diagonal entries are too small to divide by (a U3 with
    theta = pi, an X) keep the real-diagonal form, parameterised slots too;
    the others take the unit-diagonal form; the states equal the oracle's."""
    from compiled_cpu import pass_source
    rng = np.random.default_rng(21)
    n = 9
    ops = []
    for layer in range(6):
        for q in range(n):
            th = np.pi if (q + layer) % 4 == 0 else rng.uniform(0, 2 * np.pi)
            ops.append({"kind": "gate", "name": "U3", "qubits": (q,), "tag": "U3",
                        "params": (th, rng.uniform(0, 2 * np.pi), rng.uniform(0, 2 * np.pi))})
        for q in range(layer % 2, n - 1, 2):
            ops.append({"kind": "gate", "name": "CZ", "qubits": (q, q + 1), "params": (), "tag": "CZ"})
    circ = {"n_qubits": n, "ops": ops, "channels": [{"name": "depolarizing", "nq": 1, "p": 0.05}],
            "rules": [{"when": "after_tag", "tag": "U3", "channel": 0}]}
    plan = P.ptsbe_plan(circ, pair_fusion=False, tile_qubits=6)
    srcs = "".join(pass_source(plan, p) for p in range(plan.info["n_passes"]))
    assert "= cu(x0, m1, x1)" in srcs and "= cr(m0.x, x0, m1, x1)" in srcs
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=5, total_shots=5, seed=3, cfg=4)
    st = run_compiled(plan, ts)
    ref, _ = oracle_states(circ, ts.get()["records"])
    assert max(float(np.max(np.abs(st[a] - ref[a]))) for a in range(len(ref))) <= 1e-5
    hea = hea_circuit(8, 3, np.random.default_rng(4), 0.05)
    hp = P.ptsbe_plan(hea, pair_fusion=False)
    hs = "".join(pass_source(hp, p) for p in range(hp.info["n_passes"]))
    assert "= cr(m0.x, x0, m1, x1)" in hs        # parameterised rotations keep the real diagonal
