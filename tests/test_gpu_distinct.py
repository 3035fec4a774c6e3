"""Distinct shots per trajectory on the GPU (ptsbe_unique_shots) against the
oracle's `distinct`, value for value and count for count: sampler output of
the 10-qubit workload, synthetic shot buffers with heavy repetition, zero-shot
trajectories, trajectories spanning many sampler chunks, 64-bit shot words
(n > 32) and workspaces that force one or a few trajectories per batch."""

import numpy as np
import pytest
import torch

import paper_2504_16297_amd as P
from gpu_helpers import log
from oracle.sampling import distinct
from workloads import c1_workload

pytestmark = pytest.mark.gpu


def _check(ts, bits_dev, m, **kw):
    r = P.ptsbe_unique_shots(ts, bits_dev, pairs=True, **kw)
    torch.cuda.synchronize()
    uniq = r["unique"].cpu().numpy()
    idx = r["index"].cpu().numpy().astype(np.int64)
    cnt = r["count"].cpu().numpy().astype(np.int64)
    bits = bits_dev.cpu().numpy().astype(np.int64)
    off = np.concatenate([[0], np.cumsum(m)]).astype(np.int64)
    for a in range(len(m)):
        v, c = distinct(bits[off[a]:off[a + 1]])
        assert uniq[a] == len(v), f"trajectory {a}"
        assert np.array_equal(idx[off[a]:off[a] + len(v)], v), f"trajectory {a}"
        assert np.array_equal(cnt[off[a]:off[a] + len(v)], c), f"trajectory {a}"
    return uniq


def test_sampler_output_of_c1():
    wl = c1_workload()
    plan = P.ptsbe_plan(wl["circuit"], precision="c128")
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=64, total_shots=64000, seed=0, cfg=1)
    s = P.ptsbe_run_batch(plan, ts, mode="shots", seed=0, cfg=1)
    m = ts.get()["m"]
    uniq = _check(ts, s["bits"], m)
    log(f"[distinct c1] {len(m)} trajectories, mean unique fraction {np.mean(uniq / np.maximum(m, 1)):.3f}")


@pytest.mark.parametrize("max_batch", [0, 1, 3])
def test_synthetic_repetition_zero_shots_and_batches(max_batch):
    circ = {"n_qubits": 10, "ops": [{"kind": "gate", "name": "H", "qubits": (0,), "params": ()}],
            "channels": [], "rules": [], "params": []}
    plan = P.ptsbe_plan(circ)
    m = np.array([5, 0, 3000, 1, 0, 20000, 64, 7], dtype=np.uint64)
    ts = P.ptsbe_trajset_from_records(plan, [()] * len(m), m)
    rng = np.random.default_rng(11)
    # few distinct values: long repeated runs across sampler-sized chunks
    bits = np.concatenate([rng.integers(0, 1 << int(rng.integers(1, 11)), size=int(k)) for k in m])
    log(f"[distinct synthetic] max_batch={max_batch} shots={bits.size}")
    _check(ts, torch.tensor(bits.astype(np.int32), device="cuda"), m, max_batch=max_batch)


def test_64_bit_shot_words():
    circ = {"n_qubits": 34, "ops": [{"kind": "gate", "name": "H", "qubits": (33,), "params": ()}],
            "channels": [], "rules": [], "params": []}
    plan = P.ptsbe_plan(circ)
    m = np.array([9000, 1, 4097], dtype=np.uint64)
    ts = P.ptsbe_trajset_from_records(plan, [()] * len(m), m)
    rng = np.random.default_rng(5)
    pool = rng.integers(0, 1 << 34, size=600)
    bits = pool[rng.integers(0, pool.size, size=int(m.sum()))]
    _check(ts, torch.tensor(bits.astype(np.int64), device="cuda"), m)
