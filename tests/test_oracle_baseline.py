"""Pins of the conventional per-shot baseline (Algorithm 1)."""

import numpy as np

from oracle.baseline import STREAM_BASELINE, per_shot
from oracle.densitymatrix import outcome_distribution
from oracle.noise import expand, site_channels, site_probs
from oracle.pts import proportional
from oracle.sampling import sample
from oracle.statevector import run_record
from workloads import random_small_circuit


def test_interleaved_draws_equal_pre_drawn_records():
    """Drawing each site's operator during the walk (Algorithm 1) or before it
    (PTS with one shot per draw, on the same stream) gives the same shots."""
    circ = random_small_circuit(4, 20, np.random.default_rng(2), p1=0.2, p2=0.3)
    shots, recs = per_shot(circ, 40, 3, 1)
    sp = site_probs(circ)
    pre, _ = proportional(sp, 3, 1, 40, stream=STREAM_BASELINE, merge=False)
    assert list(recs) == list(pre)
    ss = expand(circ)
    ch = site_channels(circ)
    for i, rec in enumerate(pre):
        psi, _ = run_record(circ, rec, steps_sites=ss, chans=ch)
        idx, _ = sample(psi, 1, 3, 1, i)
        assert idx[0] == shots[i]


def test_per_shot_histogram_matches_channel():
    circ = random_small_circuit(3, 8, np.random.default_rng(6), p1=0.2, p2=0.3)
    exact = outcome_distribution(circ)
    n = 1500
    shots, _ = per_shot(circ, n, 11, 1)
    hist = np.bincount(shots, minlength=exact.size) / n
    tvd = 0.5 * np.sum(np.abs(hist - exact))
    # 8 outcomes at 1500 shots: the expected TVD is about 0.03
    assert tvd < 0.08
