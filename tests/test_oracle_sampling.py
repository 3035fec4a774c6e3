"""Pins of the oracle's shot sampler against |psi|^2 and the upper-bound rule."""

import math

import numpy as np

from oracle.gates import gate_matrix, u3
from oracle.sampling import boundary_distance, cdf, chunk_sorted, draw, sample
from oracle.statevector import apply, zero_state


def _rand_state(rng, n):
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


def chi2_merged(counts, probs, min_expected=5.0):
    """Pearson statistic and degrees of freedom after merging bins (in index order)
    until each has an expected count of at least ``min_expected``."""
    n = counts.sum()
    stat = 0.0
    dof = -1
    acc_c = acc_e = 0.0
    for c, p in zip(counts, probs):
        acc_c += c
        acc_e += p * n
        if acc_e >= min_expected:
            stat += (acc_c - acc_e) ** 2 / acc_e
            dof += 1
            acc_c = acc_e = 0.0
    if acc_e > 0:
        stat += (acc_c - acc_e) ** 2 / max(acc_e, 1e-300)
        dof += 1
    return stat, dof


def test_sampler_chi_square_against_born_rule():
    rng = np.random.default_rng(5)
    n = 7
    psi = _rand_state(rng, n)
    m = 30000
    idx, _ = sample(psi, m, 1, 2, 3, chunk=4096)
    counts = np.bincount(idx, minlength=1 << n)
    p = np.abs(psi) ** 2
    stat, dof = chi2_merged(counts, p)
    # mean dof, sd sqrt(2 dof): 6 sd margin
    assert stat < dof + 6 * math.sqrt(2 * dof)


def test_zero_probability_outcomes_never_drawn():
    n = 4
    psi = zero_state(n)
    psi = apply(psi, n, gate_matrix("H"), (1,))
    psi = apply(psi, n, u3(1.0, 0.3, 0.2), (3,))
    idx, _ = sample(psi, 5000, 9, 9, 0)
    p = np.abs(psi) ** 2
    assert np.all(p[idx] > 0)
    # u = 0 selects the first outcome with nonzero probability
    c = cdf(psi)
    assert draw(c, np.array([0.0]))[0] == int(np.flatnonzero(p > 0)[0])


def test_chunk_order_and_ragged_tail():
    rng = np.random.default_rng(1)
    u = rng.random(10000)
    s = chunk_sorted(u, 4096)
    for a in range(0, 10000, 4096):
        blk = s[a:a + 4096]
        assert np.all(np.diff(blk) >= 0)
        assert np.array_equal(np.sort(u[a:a + 4096]), blk)


def test_draw_is_monotone_in_u_and_boundary_distance():
    rng = np.random.default_rng(2)
    psi = _rand_state(rng, 6)
    c = cdf(psi)
    u = np.sort(rng.random(2000))
    idx = draw(c, u)
    assert np.all(np.diff(idx) >= 0)
    d = boundary_distance(c, u)
    assert np.all(d >= 0) and np.all(d < 1)
    # each u lies in [CDF[idx-1], CDF[idx]) of the normalised CDF
    cn = c / c[-1]
    lo = np.where(idx > 0, cn[np.maximum(idx - 1, 0)], 0.0)
    assert np.all(u >= lo - 1e-15) and np.all(u < cn[idx] + 1e-15)
