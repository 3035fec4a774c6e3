"""Write the oracle-generated expected values stored under tests/golden/.

Every value written here comes from the FP64 oracle (``oracle/``) on the
seeded workload descriptions (``workloads/``); nothing is read from the HIP
library.  Run from the repository root:

    python tests/golden/make_golden.py c4      # 24-qubit brick trajectory (a few minutes)
    python tests/golden/make_golden.py c5      # 16-qubit ensemble gradient (uses all cores)

c4_24q_trajectory.npz -- the first trajectory with at least one error of the
24-qubit, 30-layer brick workload (p2 = 1e-2, 256 proportional draws sharing
2.56e7 shots, seed 0): its record, amplitudes of the normalised state at
16384 random basis indices plus the 256 largest, the squared norm of each
consecutive block of 4096 amplitudes, its first 8192 shots with the
distance of each sorted uniform to the nearest CDF boundary (Sec. 3: all
m_alpha shots drawn from one prepared state), and 1024 bins of about equal
probability (basis-index edges where the CDF crosses j / 1024, with each
bin's exact probability) for the histogram distance of all its shots.

c5_ensemble_gradient.npz -- E(theta) = sum_alpha w_alpha <psi_alpha|O|psi_alpha>
with w_alpha = count_alpha / T over the oracle's own proportional records of
the 16-qubit, 8-layer hardware-efficient ansatz (1024 draws, p2 = 5e-3,
O = sum_i Z_i Z_(i+1 mod 16)), and its gradient over the 256 parameters by the
oracle's adjoint sweep (pinned there against the parameter-shift rule).
"""

import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

C4_FILE = os.path.join(HERE, "c4_24q_trajectory.npz")
C5_FILE = os.path.join(HERE, "c5_ensemble_gradient.npz")


def make_c4():
    from oracle.noise import expand, site_channels, site_probs
    from oracle.pts import sample_kraus
    from oracle.sampling import boundary_distance, cdf, sample
    from oracle.statevector import run_record
    from workloads import c4_workload

    wl = c4_workload(24)
    circ = wl["circuit"]
    ref = sample_kraus(site_probs(circ), wl["pts"], wl["seed"], wl["cfg"])
    alpha = next(a for a, r in enumerate(ref["records"]) if len(r) > 0)
    rec = ref["records"][alpha]
    t0 = time.perf_counter()
    psi, _ = run_record(circ, rec, steps_sites=expand(circ), chans=site_channels(circ))
    print(f"c4: trajectory {alpha} ({len(rec)} errors) prepared in {time.perf_counter() - t0:.0f} s")
    w = psi.real ** 2 + psi.imag ** 2
    psi = psi / math.sqrt(math.fsum(w))
    n = circ["n_qubits"]
    rng = np.random.default_rng(24)
    idx = rng.choice(1 << n, size=16384, replace=False)
    top = np.argsort(-np.abs(psi))[:256]
    idx = np.unique(np.concatenate([idx, top])).astype(np.int64)
    prob = psi.real ** 2 + psi.imag ** 2
    block = prob.reshape(-1, 4096).sum(axis=1)
    m = int(ref["m"][alpha])
    shots, us = sample(psi, m, wl["seed"], wl["cfg"], alpha)
    k = min(8192, m)
    c = cdf(psi)
    dist = boundary_distance(c, us[:k])
    # bins of about equal mass: edge j = first index whose CDF reaches j / 1024
    edges = np.searchsorted(c, np.arange(1, 1024) / 1024.0 * c[-1], side="left")
    edges = np.unique(np.concatenate([[0], edges, [c.size]])).astype(np.int64)
    cum = np.concatenate([[0.0], c])
    bin_mass = (cum[edges[1:]] - cum[edges[:-1]]) / c[-1]
    np.savez_compressed(C4_FILE, alpha=np.int64(alpha), m=np.int64(m),
                        rec_site=np.array([s for s, _ in rec], dtype=np.int64),
                        rec_kraus=np.array([kk for _, kk in rec], dtype=np.int64),
                        amp_index=idx, amp=psi[idx], block_prob=block,
                        shots=shots[:k].astype(np.int64), boundary_distance=dist,
                        bin_edges=edges, bin_mass=bin_mass)
    print(f"c4: wrote {C4_FILE} (m = {m}, {idx.size} amplitudes, {k} shots)")


_C5 = None


def _one_thread():
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)


def _c5_one(a):
    from oracle.adjoint import trajectory_grad
    circ, recs, params, odiag, ss, ch = _C5
    return trajectory_grad(circ, recs[a], params, odiag, ss, ch)


def make_c5(procs=None):
    global _C5
    from oracle.adjoint import observable_diag
    from oracle.noise import expand, site_channels, site_probs
    from oracle.pts import sample_kraus
    from workloads import c5_workload

    wl = c5_workload()
    circ = wl["circuit"]
    params = np.asarray(circ["params"], dtype=np.float64)
    ref = sample_kraus(site_probs(circ), wl["pts"], wl["seed"], wl["cfg"])
    counts = np.asarray(ref["counts"], dtype=np.float64)
    T = float(wl["pts"]["n_draws"])
    odiag = observable_diag(circ["n_qubits"], wl["observable"])
    _C5 = (circ, ref["records"], params, odiag, expand(circ), site_channels(circ))
    procs = procs or os.cpu_count() or 1
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs, initializer=_one_thread) as pool:
        res = pool.map(_c5_one, range(len(ref["records"])), chunksize=4)
    # fixed summation order: trajectory order
    E = 0.0
    G = np.zeros(params.size)
    for (e, g), c in zip(res, counts):
        E += (c / T) * e
        G += (c / T) * g
    print(f"c5: {len(res)} trajectories in {time.perf_counter() - t0:.0f} s; E = {E:.12f}, |G| = "
          f"{np.linalg.norm(G):.6e}")
    np.savez_compressed(C5_FILE, E=np.float64(E), grad=G, counts=counts, n_draws=np.int64(T),
                        n_traj=np.int64(len(res)))
    print(f"c5: wrote {C5_FILE}")


if __name__ == "__main__":
    which = sys.argv[1:] or ["c4", "c5"]
    if "c5" in which:
        make_c5()
    if "c4" in which:
        make_c4()
