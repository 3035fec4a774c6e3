"""GPU parity of two configurations against the FP64 oracle.

* The conventional per-shot trajectories of Algorithm 1 (Sec. 2.2) on the
  10-qubit brick workload: the library's per-shot mode (one undeduplicated
  draw per shot on the baseline stream, one full state preparation per shot:
  prefix sharing off) against oracle.baseline.per_shot, shot for shot.
* One trajectory of the 24-qubit, 30-layer brick workload with errors,
  prepared and sampled exactly as the mixed-size batch runs it, against the
  oracle values tests/golden/make_golden.py stored: amplitudes at 16640 basis
  indices, squared norms of all 4096-amplitude blocks, and its first 8192
  shots (equal except where the uniform lies within 1e-6 of a CDF boundary).
"""

import math
import os

import numpy as np
import pytest
import torch

import paper_2504_16297_amd as P
from gpu_helpers import log
from oracle.baseline import STREAM_BASELINE, per_shot
from oracle.noise import expand, site_channels, site_probs
from oracle.pts import proportional
from oracle.sampling import boundary_distance, cdf, sample
from oracle.statevector import run_record
from workloads import c1_workload, c4_workload

pytestmark = pytest.mark.gpu

GOLDEN_C4 = os.path.join(os.path.dirname(__file__), "golden", "c4_24q_trajectory.npz")


def test_per_shot_baseline_matches_algorithm_1():
    wl = c1_workload()
    circ = wl["circuit"]
    n_shots = 512
    plan = P.ptsbe_plan(circ, precision=wl["precision"])
    ts = P.ptsbe_sample_kraus(plan, "per_shot", n_draws=n_shots, seed=wl["seed"], cfg=wl["cfg"])
    g = ts.get()
    assert ts.n_traj == n_shots and list(g["m"]) == [1] * n_shots
    ref_idx, ref_recs = per_shot(circ, n_shots, wl["seed"], wl["cfg"])
    assert g["records"] == list(ref_recs)
    r = P.ptsbe_run_batch(plan, ts, mode="shots", seed=wl["seed"], cfg=wl["cfg"], prefix_sharing=False)
    torch.cuda.synchronize()
    bits = r["bits"][:n_shots].cpu().numpy().astype(np.int64)
    traj = r["traj"][:n_shots].cpu().numpy()
    assert np.array_equal(traj, np.arange(n_shots))
    bad = np.flatnonzero(bits != ref_idx)
    ss, ch = expand(circ), site_channels(circ)
    unexcused = 0
    for i in bad:
        psi, _ = run_record(circ, ref_recs[i], steps_sites=ss, chans=ch)
        _, u = sample(psi, 1, wl["seed"], wl["cfg"], int(i))
        if boundary_distance(cdf(psi), u)[0] >= 1e-6:
            unexcused += 1
    log(f"[per-shot C1] {n_shots} shots, {bad.size} differ, {unexcused} away from a CDF boundary")
    assert unexcused == 0
    # with prefix sharing the same shots come out (the error-free passes are shared)
    r2 = P.ptsbe_run_batch(plan, ts, mode="shots", seed=wl["seed"], cfg=wl["cfg"])
    torch.cuda.synchronize()
    assert np.array_equal(r2["bits"][:n_shots].cpu().numpy(), r["bits"][:n_shots].cpu().numpy())


@pytest.mark.parametrize("tile", [0, 13])
def test_c4_24q_trajectory_against_oracle(tile):
    """One 24-qubit trajectory of the mixed batch against stored oracle values,
    with the default 12-qubit tiles and with 13-qubit tiles (512 threads)."""
    gold = np.load(GOLDEN_C4)
    wl = c4_workload(24)
    circ = wl["circuit"]
    alpha = int(gold["alpha"])
    plan = P.ptsbe_plan(circ, precision=wl["precision"], tile_qubits=tile)
    pts = wl["pts"]
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=pts["n_draws"], total_shots=pts["total_shots"],
                              seed=wl["seed"], cfg=wl["cfg"])
    g = ts.get()
    rec = g["records"][alpha]
    assert [s for s, _ in rec] == list(gold["rec_site"]) and [k for _, k in rec] == list(gold["rec_kraus"])
    assert len(rec) >= 1 and int(g["m"][alpha]) == int(gold["m"])
    one = ts.slice(alpha, alpha + 1)          # keeps the global id: same sampler stream
    st = P.ptsbe_run_batch(plan, one, mode="states")
    torch.cuda.synchronize()
    psi = st["states"][0]
    idx = torch.as_tensor(gold["amp_index"], device=psi.device)
    amp = psi[idx].cpu().numpy().astype(np.complex128)
    err = float(np.max(np.abs(amp - gold["amp"])))
    prob = (psi.real.double() ** 2 + psi.imag.double() ** 2).reshape(-1, 4096).sum(dim=1).cpu().numpy()
    berr = float(np.max(np.abs(prob - gold["block_prob"])))
    del st, psi
    sh = P.ptsbe_run_batch(plan, one, mode="shots", seed=wl["seed"], cfg=wl["cfg"])
    torch.cuda.synchronize()
    k = gold["shots"].size
    bits = sh["bits"][:k].cpu().numpy().astype(np.int64)
    bad = np.flatnonzero(bits != gold["shots"])
    unexcused = int(np.sum(gold["boundary_distance"][bad] >= 1e-6))
    log(f"[C4 24q] trajectory {alpha} ({len(rec)} errors): max|amp err| {err:.2e} over {idx.numel()} "
        f"amplitudes, block mass err {berr:.2e}, {bad.size} of {k} shots differ ({unexcused} unexcused)")
    assert err <= 1e-5
    assert berr <= 1e-6
    assert unexcused == 0
    assert math.isclose(float(prob.sum()), 1.0, abs_tol=1e-6)


def test_per_shot_draws_are_the_baseline_stream():
    """The per-shot mode's records are proportional draws on the baseline
    stream, one per shot, not merged (host check, run here beside the GPU
    comparison above)."""
    wl = c1_workload()
    plan = P.ptsbe_plan(wl["circuit"], precision=wl["precision"])
    ts = P.ptsbe_sample_kraus(plan, "per_shot", n_draws=64, seed=wl["seed"], cfg=wl["cfg"])
    recs, _ = proportional(site_probs(wl["circuit"]), wl["seed"], wl["cfg"], 64, stream=STREAM_BASELINE,
                           merge=False)
    assert ts.get()["records"] == recs
