"""The 20-qubit, 40-layer brick workload at its full size, in the launch
configuration bench.py times (complex64 plan, compiled passes, prefix sharing,
one run of all 480 trajectories and 10^6 shots into caller buffers): shot
bookkeeping over the whole job, and for sampled trajectories (the first and the
one with the most errors) the shots against the oracle's sampler on the
oracle's complex128 state, plus their amplitudes."""

import numpy as np
import pytest
import torch

import paper_2504_16297_amd as P
from gpu_helpers import compare_shots, log, oracle_states
from workloads import c2_workload

pytestmark = pytest.mark.gpu


def test_c2_full_size_in_bench_configuration():
    wl = c2_workload()
    circ, pts = wl["circuit"], wl["pts"]
    plan = P.ptsbe_plan(circ, precision=wl["precision"])
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=pts["n_draws"], total_shots=pts["total_shots"],
                              seed=wl["seed"], cfg=wl["cfg"])
    g = ts.get()
    S = int(g["total_shots"])
    ws = torch.empty(P.ptsbe_workspace_size(plan, ts, mode="shots"), dtype=torch.uint8, device="cuda")
    out = {"bits": torch.empty(S, dtype=torch.int32, device="cuda"),
           "traj": torch.empty(S, dtype=torch.int32, device="cuda")}
    P.ptsbe_run_batch(plan, ts, mode="shots", seed=wl["seed"], cfg=wl["cfg"], workspace=ws, out=out)
    torch.cuda.synchronize()
    bits = out["bits"].cpu().numpy().astype(np.int64)
    traj = out["traj"].cpu().numpy().astype(np.int64)
    del ws, out
    m = np.asarray(g["m"], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(m)])
    log(f"[c2 full size] {len(m)} trajectories, {S} shots")
    assert S == pts["total_shots"] == int(m.sum())
    assert np.all((bits >= 0) & (bits < (1 << 20)))
    assert np.array_equal(traj, np.repeat(np.arange(len(m)), m))
    picks = sorted({0, int(np.argmax([len(r) for r in g["records"]]))})
    refs, _ = oracle_states(circ, [g["records"][a] for a in picks])
    for a, psi in zip(picks, refs):
        bad, excused = compare_shots(psi, bits[off[a]:off[a + 1]], int(m[a]), wl["seed"], wl["cfg"], a)
        log(f"  trajectory {a} ({len(g['records'][a])} errors, {m[a]} shots): {bad} mismatches, "
            f"{excused} within 1e-6 of a CDF boundary")
        assert bad == 0
    sub = P.ptsbe_trajset_from_records(plan, [g["records"][a] for a in picks], [1] * len(picks))
    st = P.ptsbe_run_batch(plan, sub, mode="states")["states"].cpu().numpy()
    for j, psi in enumerate(refs):
        err = float(np.max(np.abs(st[j].astype(np.complex128) - psi)))
        log(f"  trajectory {picks[j]}: max amplitude error {err:.2e}")
        assert err <= 1e-5
