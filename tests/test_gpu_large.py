"""Large-state parity (24-35 qubits), where the full oracle state is out of
reach: product-state circuits whose amplitudes the oracle computes one by one
(oracle.statevector.product_factors), shot marginals against the closed form,
expectation values of Z strings against the closed form, and, for the
entangling 24/26/28-qubit brick workloads, compiled against generic kernels
and the bookkeeping of shots and trajectory tags."""

import gc
import math

import numpy as np
import pytest
import torch

import paper_2504_16297_amd as P
from gpu_helpers import log
from oracle.statevector import product_amplitudes, product_factors
from workloads import c4_workload, product_circuit

pytestmark = pytest.mark.gpu


def _marginal_check(bits, f, n, m):
    p1 = np.abs(f[:, 1]) ** 2 / (np.abs(f[:, 0]) ** 2 + np.abs(f[:, 1]) ** 2)
    worst = 0.0
    for q in range(n):
        freq = float(np.mean((bits >> q) & 1))
        sd = math.sqrt(max(p1[q] * (1 - p1[q]), 1e-12) / m)
        worst = max(worst, abs(freq - p1[q]) / sd)
    return worst


def test_product_28q_amplitudes_and_shots():
    n = 28
    circ = product_circuit(n, 4, np.random.default_rng(28), 0.02)
    plan = P.ptsbe_plan(circ)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=4, total_shots=4 * 100000, seed=7, cfg=4)
    g = ts.get()
    log(f"[28q product] trajectories={ts.n_traj} passes={plan.info['n_passes']}")
    r = P.ptsbe_run_batch(plan, ts, mode="states")
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    xs = rng.integers(0, 1 << n, size=4096)
    xs[:2] = [0, (1 << n) - 1]
    for a in range(ts.n_traj):
        f = product_factors(circ, g["records"][a])
        ref = product_amplitudes(f, xs)
        got = r["states"][a][torch.as_tensor(xs, device="cuda")].cpu().numpy().astype(np.complex128)
        err = float(np.max(np.abs(got - ref)))
        rel = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        log(f"  trajectory {a}: max|d| = {err:.2e}, relative to the largest sampled amplitude {rel:.2e}")
        assert err <= 1e-5 and rel <= 1e-4
    del r
    torch.cuda.empty_cache()
    s = P.ptsbe_run_batch(plan, ts, mode="shots", seed=7, cfg=4)
    torch.cuda.synchronize()
    bits = s["bits"].cpu().numpy().astype(np.int64)
    traj = s["traj"].cpu().numpy()
    off = np.concatenate([[0], np.cumsum(g["m"].astype(np.int64))])
    for a in range(ts.n_traj):
        seg = slice(off[a], off[a + 1])
        assert np.all(traj[seg] == a)
        z = _marginal_check(bits[seg] & ((1 << n) - 1), product_factors(circ, g["records"][a]), n, int(g["m"][a]))
        log(f"  trajectory {a}: worst single-qubit marginal deviation {z:.2f} sigma")
        assert z < 5.5


def test_product_33q_expectations_and_shots():
    """One 33-qubit trajectory (64 GiB complex64 state): Z and ZZ expectation
    values and single-qubit shot marginals against the product closed form."""
    n = 33
    circ = product_circuit(n, 2, np.random.default_rng(33), 0.0)
    plan = P.ptsbe_plan(circ)
    ts = P.ptsbe_trajset_from_records(plan, [()], [1000000])
    f = product_factors(circ, ())
    z = (np.abs(f[:, 0]) ** 2 - np.abs(f[:, 1]) ** 2)
    obs = [(1.0, (0,)), (0.5, (17, 32)), (0.25, (31,))]
    ref = 1.0 * z[0] + 0.5 * z[17] * z[32] + 0.25 * z[31]
    r = P.ptsbe_run_batch(plan, ts, mode="expectation", observable=obs)
    torch.cuda.synchronize()
    got = float(r["expval"].cpu().numpy()[0])
    log(f"[33q product] passes={plan.info['n_passes']} <O> = {got:.8f}, closed form {ref:.8f}")
    assert abs(got - ref) <= 1e-5
    del r
    torch.cuda.empty_cache()
    s = P.ptsbe_run_batch(plan, ts, mode="shots", seed=1, cfg=4)
    torch.cuda.synchronize()
    bits = s["bits"].cpu().numpy()
    assert s["bits"].dtype == torch.int64 and np.all(bits >= 0) and np.all(bits < (1 << n))
    zs = _marginal_check(bits.astype(np.int64), f, n, 1000000)
    log(f"  worst single-qubit marginal deviation {zs:.2f} sigma")
    assert zs < 5.5


def test_product_35q_on_one_gpu():
    """One 35-qubit trajectory: a 256 GiB complex64 state on one GPU (the
    paper's statevector scale, which took four 80 GB GPUs), the FP64 CDF
    written in place over it; 10^6 shots whose single-qubit marginals, and
    the <Z Z> value, match the product closed form."""
    n = 35
    circ = product_circuit(n, 2, np.random.default_rng(35), 0.0)
    plan = P.ptsbe_plan(circ)
    ts = P.ptsbe_trajset_from_records(plan, [()], [1000000])
    need = P.ptsbe_workspace_size(plan, ts, mode="shots") + 16 * 1000000
    gc.collect()                  # earlier tests' buffers: free them and return torch's cached blocks
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    log(f"[35q product] workspace {need / 2**30:.1f} GiB, device free {free / 2**30:.1f} GiB")
    if free < need + (1 << 30):
        pytest.skip("not enough device memory for a 2^35 complex64 state")
    f = product_factors(circ, ())
    s = P.ptsbe_run_batch(plan, ts, mode="shots", seed=2, cfg=4)
    torch.cuda.synchronize()
    bits = s["bits"].cpu().numpy()
    del s
    torch.cuda.empty_cache()
    assert np.all(bits >= 0) and np.all(bits < (1 << n))
    zs = _marginal_check(bits.astype(np.int64), f, n, 1000000)
    log(f"  passes={plan.info['n_passes']} worst single-qubit marginal deviation {zs:.2f} sigma")
    assert zs < 5.5
    z = (np.abs(f[:, 0]) ** 2 - np.abs(f[:, 1]) ** 2)
    obs = [(1.0, (3, 34))]
    r = P.ptsbe_run_batch(plan, ts, mode="expectation", observable=obs)
    torch.cuda.synchronize()
    got = float(r["expval"].cpu().numpy()[0])
    log(f"  <Z3 Z34> = {got:.8f}, closed form {z[3] * z[34]:.8f}")
    assert abs(got - z[3] * z[34]) <= 1e-5


@pytest.mark.parametrize("n", [24, 28])
def test_brick_compiled_vs_generic_and_tags(n):
    """The entangling brick workload: compiled and generic kernels agree on
    the states of two trajectories; every shot carries its trajectory's tag,
    in the trajectory's own m_alpha range."""
    wl = c4_workload(n)
    circ = wl["circuit"]
    pc = P.ptsbe_plan(circ)
    pg = P.ptsbe_plan(circ, compile=False)
    ts = P.ptsbe_sample_kraus(pc, "proportional", n_draws=wl["pts"]["n_draws"],
                              total_shots=wl["pts"]["total_shots"], seed=wl["seed"], cfg=wl["cfg"])
    g = ts.get()
    sub_c = ts.slice(0, 2)
    sub_g = P.ptsbe_trajset_from_records(pg, g["records"][:2], g["m"][:2])
    a = P.ptsbe_run_batch(pc, sub_c, mode="states")["states"]
    b = P.ptsbe_run_batch(pg, sub_g, mode="states")["states"]
    torch.cuda.synchronize()
    d = float((a - b).abs().max())
    nrm = float((a.abs() ** 2).sum(dim=1).max())
    log(f"[{n}q brick] compiled vs generic max|d| = {d:.2e}, max norm^2 = {nrm:.8f}")
    assert d <= 1e-6 and abs(nrm - 1) <= 1e-4
    del a, b
    torch.cuda.empty_cache()
    s = P.ptsbe_run_batch(pc, ts, mode="shots", seed=wl["seed"], cfg=wl["cfg"])
    torch.cuda.synchronize()
    traj = s["traj"].cpu().numpy()
    bits = s["bits"].cpu().numpy()
    assert np.all(bits >= 0) and np.all(bits < (1 << n))
    counts = np.bincount(traj, minlength=ts.n_traj)
    assert np.array_equal(counts, g["m"].astype(np.int64))
    assert np.all(np.diff(traj) >= 0)


def test_surface_code_billion_shots():
    """The d=3 surface-code workload at full size: top-4096 most-likely records
    sharing 10^9 shots.  Every shot's tag and count, the support of sampled
    trajectories (noiseless support XOR the trajectory's Pauli frame), and exact
    shots of a small trajectory against the oracle."""
    from gpu_helpers import compare_shots, oracle_states
    from oracle.stabilizer import frame_run
    from workloads import c3_workload
    wl = c3_workload()
    circ = wl["circuit"]
    plan = P.ptsbe_plan(circ)
    ts = P.ptsbe_sample_kraus(plan, "most_likely", k_max=4096, total_shots=10**9, seed=0, cfg=3)
    g = ts.get()
    m = g["m"].astype(np.int64)
    assert int(m.sum()) == 10**9
    r = P.ptsbe_run_batch(plan, ts, seed=0, cfg=3)
    P.ptsbe_run_status(plan, r["workspace"])
    torch.cuda.synchronize()
    bits, traj = r["bits"], r["traj"]
    counts = torch.bincount(traj.long(), minlength=ts.n_traj).cpu().numpy()
    assert np.array_equal(counts, m)
    assert bool((traj[1:] >= traj[:-1]).all())
    log(f"[C3 1e9] trajectories={ts.n_traj} largest m={m.max()}")
    psi0, _ = oracle_states(circ, [()])
    support0 = np.flatnonzero(np.abs(psi0[0]) ** 2 > 1e-12)
    off = np.concatenate([[0], np.cumsum(m)])
    for a in (0, 1, 100, 2000, 4095):
        _, xf = frame_run(circ, g["records"][a])
        allowed = set(int(s) ^ int(xf) for s in support0)
        seen = set(torch.unique(bits[off[a]:off[a + 1]]).cpu().numpy().tolist())
        assert seen <= allowed, f"trajectory {a}"
    small = int(np.argmin(np.where(m > 1000, m, np.iinfo(np.int64).max)))
    ref, _ = oracle_states(circ, [g["records"][small]])
    seg = bits[off[small]:off[small + 1]].cpu().numpy()
    bad, exc = compare_shots(ref[0], seg, int(m[small]), 0, 3, small)
    log(f"  trajectory {small}: {m[small]} shots, {bad} mismatches, {exc} excused")
    assert bad == 0
