"""ptsbe_run_batch_noalloc (through the C ABI) against ptsbe_run_batch: the
same shots, tags, states and measure-reset records from the library's fixed
device scratch instead of a caller workspace, on consecutive calls whose
inputs shrink, with batches split to fit the scratch, and a clear error for a
state that cannot fit it."""

import numpy as np
import pytest
import torch

import paper_2504_16297_amd as P
from paper_2504_16297_amd import _lib as L
from gpu_helpers import log
from workloads import random_small_circuit
from workloads.circuits import brick_circuit, surface_code_d3

pytestmark = pytest.mark.gpu

E_OOM = 5


def _shots(plan, ts, **kw):
    r = P.ptsbe_run_batch(plan, ts, mode="shots", seed=11, cfg=3, **kw)
    torch.cuda.synchronize()
    S = int(ts.get()["total_shots"])
    return r["bits"][:S].cpu().numpy(), r["traj"][:S].cpu().numpy(), r


def _states(plan, ts, **kw):
    r = P.ptsbe_run_batch(plan, ts, mode="states", **kw)
    torch.cuda.synchronize()
    return r["states"].cpu().numpy()


def _compare(plan, ts, what):
    b0, t0, _ = _shots(plan, ts)                 # loads the compiled passes on the device
    b1, t1, _ = _shots(plan, ts, noalloc=True)   # same kernels, scratch workspace
    log(f"[noalloc] {what}: {ts.n_traj} trajectories, {b0.size} shots")
    assert np.array_equal(t0, t1)
    assert np.array_equal(b0, b1)
    s0 = _states(plan, ts)
    s1 = _states(plan, ts, noalloc=True)
    assert np.array_equal(s0, s1)


def test_noalloc_matches_run_batch_on_shrinking_inputs():
    torch.cuda.set_device(0)
    # first call: 12 qubits, several 4096-amplitude tiles per state
    c12 = random_small_circuit(12, 160, np.random.default_rng(71), p1=0.05, p2=0.1)
    plan12 = P.ptsbe_plan(c12)
    ts12 = P.ptsbe_sample_kraus(plan12, "proportional", n_draws=48, total_shots=20000, seed=4, cfg=3)
    _compare(plan12, ts12, "12 qubits")
    # second call, smaller input: 7 qubits, fewer trajectories and shots
    c7 = random_small_circuit(7, 60, np.random.default_rng(72), p1=0.05, p2=0.1)
    plan7 = P.ptsbe_plan(c7)
    ts7 = P.ptsbe_sample_kraus(plan7, "proportional", n_draws=9, total_shots=700, seed=4, cfg=3)
    _compare(plan7, ts7, "7 qubits")


def test_noalloc_splits_batches_to_fit_the_scratch():
    # 20 qubits: 8 MiB per complex64 state, so the 64 MiB scratch holds a few at a time
    torch.cuda.set_device(0)
    circ = brick_circuit(20, 6, np.random.default_rng(73), 1e-3, 2e-2)
    plan = P.ptsbe_plan(circ)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=24, total_shots=50000, seed=4, cfg=3)
    assert ts.n_traj * (8 << 20) > L.NOALLOC_SCRATCH_BYTES
    b0, t0, _ = _shots(plan, ts)
    b1, t1, _ = _shots(plan, ts, noalloc=True)
    log(f"[noalloc] 20 qubits: {ts.n_traj} trajectories split over the scratch")
    assert np.array_equal(t0, t1) and np.array_equal(b0, b1)


def test_noalloc_generic_kernels_when_not_loaded():
    # a plan never run by ptsbe_run_batch: its compiled passes are not loaded,
    # so the no-allocation call runs the generic tile kernels on the same tables
    torch.cuda.set_device(0)
    circ = random_small_circuit(10, 120, np.random.default_rng(74), p1=0.05, p2=0.1)
    plan = P.ptsbe_plan(circ)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=16, total_shots=4000, seed=4, cfg=3)
    s1 = _states(plan, ts, noalloc=True)
    s0 = _states(plan, ts)
    assert float(np.max(np.abs(s0 - s1))) <= 1e-5


def test_noalloc_measure_reset_records_and_status():
    torch.cuda.set_device(0)
    circ = surface_code_d3(rounds=2)
    plan = P.ptsbe_plan(circ)
    ts = P.ptsbe_sample_kraus(plan, "most_likely", k_max=64, total_shots=64000, seed=0, cfg=3)
    b0, t0, r0 = _shots(plan, ts)
    P.ptsbe_run_status(plan, r0["workspace"])
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    b1, t1, r1 = _shots(plan, ts, noalloc=True, status=st)
    assert int(st.cpu()[0]) == 0
    assert np.array_equal(r0["mr_bits"].cpu().numpy(), r1["mr_bits"].cpu().numpy())
    assert np.array_equal(t0, t1) and np.array_equal(b0, b1)


def test_noalloc_rejects_a_state_beyond_the_scratch():
    torch.cuda.set_device(0)
    circ = {"n_qubits": 24, "ops": [{"kind": "gate", "name": "H", "qubits": (23,), "params": ()}],
            "channels": [], "rules": [], "params": []}
    plan = P.ptsbe_plan(circ)
    ts = P.ptsbe_trajset_from_records(plan, [()], [10])
    with pytest.raises(P.PtsbeError) as e:
        P.ptsbe_run_batch(plan, ts, mode="shots", noalloc=True)
    assert e.value.status == E_OOM and "MiB" in str(e.value)
