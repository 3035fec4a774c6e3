"""Pins of the oracle's pre-trajectory sampling (Sec. 3.1) and its random streams."""

import math

import numpy as np
import pytest

from oracle import rng as orng
from oracle.pts import (_categorical, alg2_draw, allocate_multiplicity, allocate_reweight,
                        joint_prob, most_likely, most_likely_bruteforce, proportional, score,
                        costs)

# --- Philox4x64-10 written out from the published description (Salmon et al., SC'11):
# two 64x64->128 multiplies per round, Weyl key schedule, 10 rounds.
M0, M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
W0, W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B
MASK = (1 << 64) - 1


def _philox_block(ctr, key):
    c = list(ctr)
    k = list(key)
    for r in range(10):
        if r:
            k = [(k[0] + W0) & MASK, (k[1] + W1) & MASK]
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k[0], p1 & MASK, (p0 >> 64) ^ c[3] ^ k[1], p0 & MASK]
    return c


@pytest.mark.parametrize("key", [(0, 0), (0, orng.key1(2, 3, 17)), (12345, orng.key1(1, 5, 999)),
                                 (2**63 + 5, 2**64 - 1)])
def test_philox_stream_matches_published_definition(key):
    w = orng.words(key[0], key[1], 13)
    for j in range(13):
        # word j of a stream is word j % 4 of the block with counter j // 4 + 1
        assert int(w[j]) == _philox_block([j // 4 + 1, 0, 0, 0], key)[j % 4]


def test_uniform_construction():
    w = orng.words(7, 9, 8)
    u = orng.uniforms(7, 9, 8)
    for a, b in zip(w, u):
        assert b == (int(a) >> 11) / 2.0**53
        assert 0.0 <= b < 1.0


def test_categorical_upper_bound_rule():
    p = [0.5, 0.25, 0.25]
    assert _categorical(0.0, p) == 0
    assert _categorical(0.4999999, p) == 0
    assert _categorical(0.5, p) == 1
    assert _categorical(0.7499999, p) == 1
    assert _categorical(0.75, p) == 2
    assert _categorical(1.0 - 2.0**-53, p) == 2
    assert _categorical(0.3, [0.0, 1.0]) == 1      # zero-probability index never selected


def _chi2_ok(counts, probs, n, thresh=40.0):
    """Pearson statistic small for 3-4 bins (p-value far from tiny)."""
    exp = np.asarray(probs) * n
    return float(np.sum((np.asarray(counts) - exp) ** 2 / exp)) < thresh


def test_proportional_per_site_frequencies():
    sp = [[0.7, 0.1, 0.1, 0.1], [0.6, 0.4], [0.5, 0.2, 0.2, 0.1]]
    T = 6000
    recs, cnt = proportional(sp, 4, 1, T, merge=False)
    for s, probs in enumerate(sp):
        c = np.zeros(len(probs))
        for rec in recs:
            c[dict(rec).get(s, 0)] += 1
        assert _chi2_ok(c, probs, T)


def test_alg2_literal_closed_form_bias():
    """Algorithm 2 as printed on a 1q depolarizing site: P(X) = q, P(Y) = (1-q) q,
    P(Z) = (1-q)^2 q, P(none) = (1-q)^3 with q = p/3 -- not the channel's p/3 each."""
    p = 0.45
    q = p / 3
    sp = [[1 - p, q, q, q]]
    T = 8000
    c = np.zeros(4)
    for t in range(T):
        rec = alg2_draw(sp, 2, 1, t)
        c[dict(rec).get(0, 0)] += 1
    expect = [(1 - q) ** 3, q, (1 - q) * q, (1 - q) ** 2 * q]
    assert _chi2_ok(c, expect, T)
    # the bias against the channel's own probabilities is visible at this size
    assert not _chi2_ok(c, sp[0], T, thresh=100.0)


def test_multiplicity_allocation_by_hand():
    assert allocate_multiplicity([3, 1], 4, 10) == [8, 2]
    assert allocate_multiplicity([1, 1, 1], 3, 10) == [4, 3, 3]
    assert allocate_multiplicity([2, 1, 1], 4, 1000) == [500, 250, 250]
    m = allocate_multiplicity([5, 3, 2, 1, 1], 12, 10**6 + 7)
    assert sum(m) == 10**6 + 7


def test_reweight_allocation_by_hand():
    assert allocate_reweight([0.5, 0.25, 0.25], 8) == [4, 2, 2]
    assert allocate_reweight([0.2, 0.2, 0.2], 10) == [4, 3, 3]
    m = allocate_reweight([0.3, 1e-9, 0.1, 0.05], 10**9)
    assert sum(m) == 10**9


def test_joint_probability_product():
    sp = [[0.9, 0.1], [0.8, 0.05, 0.15]]
    assert joint_prob((), sp) == 0.9 * 0.8
    assert joint_prob(((1, 2),), sp) == 0.9 * 0.15
    assert joint_prob(((0, 1), (1, 1)), sp) == 0.1 * 0.05


@pytest.mark.parametrize("seed", range(6))
def test_most_likely_matches_exhaustive_sort(seed):
    rng = np.random.default_rng(seed)
    n_sites = int(rng.integers(3, 9))
    proto = [[1 - 0.1, 0.1 / 3, 0.1 / 3, 0.1 / 3], [0.8, 0.2], [0.7, 0.1, 0.15, 0.05]]
    sp = [proto[int(rng.integers(3))] for _ in range(n_sites)]   # repeated types -> exact ties
    total = int(np.prod([len(p) for p in sp]))
    for K in (1, 5, 17, min(200, total), total):
        r1, s1 = most_likely(sp, K)
        r2, s2 = most_likely_bruteforce(sp, K)
        assert r1 == r2
        assert s1 == s2


def test_score_is_order_canonical():
    sp = [[0.9, 0.1], [0.9, 0.1], [0.8, 0.2]]
    c = costs(sp)
    assert score(((0, 1), (2, 1)), c) == score(((1, 1), (2, 1)), c)
    assert math.isclose(score(((0, 1),), c), -math.log(0.1 / 0.9))


def _small_probs(seed, S=7):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(S):
        K = int(rng.integers(2, 5))
        p = rng.dirichlet(np.full(K, 0.6))
        p = np.sort(p)[::-1]
        out.append(p)
    return out


@pytest.mark.parametrize("seed", range(4))
def test_most_likely_with_criteria_matches_exhaustive_sort(seed):
    from oracle.pts import most_likely_bruteforce
    sp = _small_probs(100 + seed)
    allow = {(s, k) for s in range(len(sp)) for k in range(1, len(sp[s])) if (s + k + seed) % 3}
    for crit in ({}, {"min_errors": 2}, {"max_errors": 2}, {"parity": "odd"}, {"parity": "even", "min_errors": 1}):
        for a in (None, allow):
            r1, s1 = most_likely(sp, 9, allow=a, **crit)
            r2, s2 = most_likely_bruteforce(sp, 9, allow=a, **crit)
            assert r1 == r2 and s1 == s2, (crit, a is None)


def test_selection_special_cases():
    from oracle.pts import select_records
    sp = _small_probs(7)
    every = {(s, k) for s in range(len(sp)) for k in range(1, len(sp[s]))}
    base = proportional(sp, 3, 1, 200)
    assert proportional(sp, 3, 1, 200, allow=every) == base        # allowing all changes nothing
    recs, counts = proportional(sp, 3, 1, 200, allow=set())
    assert recs == [()] and counts == [200]                        # allowing none: the error-free record
    # an operator outside `allow` maps to operator 0, draw by draw
    drop = {(0, 1), (3, 1)}
    r_all, _ = proportional(sp, 3, 1, 200, merge=False)
    r_sel, _ = proportional(sp, 3, 1, 200, merge=False, allow=every - drop)
    assert r_sel == [tuple(x for x in r if x not in drop) for r in r_all]
    # record filters drop whole records with their draws
    kept, kc = select_records(base[0], base[1], parity="odd", max_errors=3)
    assert all(len(r) % 2 == 1 and len(r) <= 3 for r in kept)
    assert sum(kc) == sum(c for r, c in zip(*base) if len(r) % 2 == 1 and len(r) <= 3)


# --- probability band (Sec. 3.1: a Kraus operator set is chosen only if p_alpha lies in [p_min, p_max])

_BAND_SP = [[0.9, 0.1], [0.8, 0.15, 0.05]]
# every record of _BAND_SP with its joint probability, worked out by hand
_BAND_ALL = [((), 0.72), (((0, 1),), 0.08), (((1, 1),), 0.135), (((1, 2),), 0.045),
             (((0, 1), (1, 1)), 0.015), (((0, 1), (1, 2)), 0.005)]


def test_probability_band_by_hand():
    from oracle.pts import probability_band
    recs = [r for r, _ in _BAND_ALL]
    counts = [50, 9, 13, 5, 2, 1]
    kr, kc, T = probability_band(recs, counts, _BAND_SP, 0.01, 0.1)
    assert kr == [((0, 1),), ((1, 2),), ((0, 1), (1, 1))]
    assert kc == [9, 5, 2] and T == 16
    # multiplicity over the kept draws: 900/16, 500/16, 200/16 = 56.25, 31.25, 12.5;
    # the one shot left goes to the largest remainder (200 mod 16 = 8)
    assert allocate_multiplicity(kc, T, 100) == [56, 31, 13]
    # reweight over the kept set: p' = (0.08, 0.045, 0.015) / 0.14 of 1000 shots
    # = 571.43, 321.43, 107.14 -> 571, 321, 107 and the last shot to the first (ties to lower alpha)
    assert allocate_reweight([joint_prob(r, _BAND_SP) for r in kr], 1000) == [572, 321, 107]


def test_probability_band_edges():
    from oracle.pts import probability_band
    recs = [r for r, _ in _BAND_ALL]
    ps = [joint_prob(r, _BAND_SP) for r in recs]
    counts = [1] * len(recs)
    # both ends are included: a band of one value keeps exactly the records of that probability
    for r, p in zip(recs, ps):
        kr, _, _ = probability_band(recs, counts, _BAND_SP, p, p)
        assert kr == [x for x, q in zip(recs, ps) if q == p] and r in kr
    # [0, 1] keeps everything; a band between the probabilities keeps nothing
    assert probability_band(recs, counts, _BAND_SP, 0.0, 1.0)[0] == recs
    assert probability_band(recs, counts, _BAND_SP, 0.2, 0.7)[0] == []


def test_probability_band_draws_follow_the_conditional_distribution():
    """Proportional draws restricted to a band: the kept records appear with
    p_alpha / P(band), the channel's distribution conditioned on the band."""
    from oracle.pts import probability_band
    T = 20000
    recs, counts = proportional(_BAND_SP, 11, 1, T)
    kr, kc, Tk = probability_band(recs, counts, _BAND_SP, 0.01, 0.2)
    inband = [(r, p) for r, p in _BAND_ALL if 0.01 <= p <= 0.2]
    pb = sum(p for _, p in inband)
    got = dict(zip(kr, kc))
    obs = [got.get(r, 0) for r, _ in inband]
    assert sum(obs) == Tk
    assert _chi2_ok(obs, [p / pb for _, p in inband], Tk)
    # and the kept fraction of the draws is P(band) = 0.08 + 0.135 + 0.045 + 0.015
    assert abs(Tk / T - pb) < 4 * math.sqrt(pb * (1 - pb) / T)


def test_sample_kraus_band_composes_sampler_band_and_allocation():
    from oracle.pts import probability_band, sample_kraus
    sp = _small_probs(3, S=6)
    for pts in ({"mode": "proportional", "n_draws": 300, "total_shots": 5000, "alloc": "multiplicity"},
                {"mode": "most_likely", "k_max": 40, "total_shots": 5000, "alloc": "reweight"},
                {"mode": "alg2_literal", "n_draws": 300, "nshots": 7, "alloc": "uniform"}):
        full = sample_kraus(sp, pts, 5, 2)
        ps = sorted(full["p"])
        band = (ps[len(ps) // 4], ps[3 * len(ps) // 4])
        got = sample_kraus(sp, dict(pts, p_band=band), 5, 2)
        kr, kc, T = probability_band(full["records"], full["counts"], sp, *band)
        assert got["records"] == kr and got["counts"] == kc
        assert all(band[0] <= p <= band[1] for p in got["p"])
        if pts["alloc"] == "multiplicity":
            assert got["m"] == allocate_multiplicity(kc, T, 5000) and sum(got["m"]) == 5000
        elif pts["alloc"] == "reweight":
            assert got["m"] == allocate_reweight(got["p"], 5000)
        else:
            assert got["m"] == [7] * len(kr)
