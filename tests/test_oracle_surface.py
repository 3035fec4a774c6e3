"""Pins of the oracle's measure-reset (general Kraus branch of Algorithm 1) on the
d=3 surface-code memory workload, against Pauli-frame propagation."""

import numpy as np
import pytest

from oracle.noise import expand, site_channels, site_probs
from oracle.pts import most_likely, proportional
from oracle.stabilizer import frame_run
from oracle.statevector import run_record
from workloads import c3_workload
from workloads.circuits import SURFACE_D3_CHECKS


@pytest.fixture(scope="module")
def c3():
    wl = c3_workload()
    circ = wl["circuit"]
    return circ, expand(circ), site_channels(circ), site_probs(circ)


def test_stabilisers_commute():
    for ka, sa in SURFACE_D3_CHECKS:
        for kb, sb in SURFACE_D3_CHECKS:
            if ka != kb:
                assert len(set(sa) & set(sb)) % 2 == 0


def test_site_and_measure_counts(c3):
    circ, (steps, sites), _, _ = c3
    assert len(sites) == 209
    assert sum(1 for s in steps if s[0] == "mr") == 40


def test_noiseless_syndromes_are_zero_and_logical_zero(c3):
    circ, ss, ch, _ = c3
    psi, bits = run_record(circ, (), steps_sites=ss, chans=ch)
    assert bits == [0] * 40
    p = np.abs(psi) ** 2
    support = np.flatnonzero(p > 1e-12)
    assert support.size == 16                    # span of the 4 X-type checks on data
    assert np.allclose(p[support], 1 / 16, atol=1e-12)
    assert np.all(support < (1 << 9))            # ancillas reset to |0>


def test_measure_reset_records_match_pauli_frames(c3):
    circ, ss, ch, sp = c3
    recs_ml, _ = most_likely(sp, 60)
    recs_p, _ = proportional(sp, 0, 3, 4)
    rng = np.random.default_rng(0)
    # a few random multi-error records too
    extra = []
    for _ in range(3):
        picks = rng.choice(len(sp), size=3, replace=False)
        extra.append(tuple(sorted((int(s), int(rng.integers(1, len(sp[s])))) for s in picks)))
    psi0, _ = run_record(circ, (), steps_sites=ss, chans=ch)
    support0 = set(np.flatnonzero(np.abs(psi0) ** 2 > 1e-12).tolist())
    for rec in recs_ml[::12] + recs_p + extra:
        psi, bits = run_record(circ, rec, steps_sites=ss, chans=ch)
        fbits, mask = frame_run(circ, rec)
        assert bits == fbits
        support = set(np.flatnonzero(np.abs(psi) ** 2 > 1e-12).tolist())
        assert support == {s ^ mask for s in support0}


def test_most_likely_selection_structure(c3):
    """Top-4096: the empty record, all 1969 single errors, then double errors."""
    _, _, _, sp = c3
    recs, scores = most_likely(sp, 4096)
    assert recs[0] == ()
    sizes = [len(r) for r in recs]
    assert sizes.count(1) == sum(len(p) - 1 for p in sp) == 1969
    assert sizes.count(2) == 4096 - 1 - 1969
    assert all(np.diff(scores) >= 0)
