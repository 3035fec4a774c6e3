"""Pins of the oracle's distinct-shot count (Sec. 4, Fig. 4's unique fraction):
hand-worked lists, the coupon-collector expectation against Monte Carlo, and
its limits (one draw, point mass, many draws)."""

import math

import numpy as np

from oracle.sampling import distinct, expected_distinct, sample


def test_hand_worked_lists():
    v, c = distinct([3, 1, 3, 2, 1, 3])
    assert v.tolist() == [3, 1, 2] and c.tolist() == [3, 2, 1]
    v, c = distinct([])
    assert v.size == 0 and c.size == 0
    v, c = distinct([7] * 5)
    assert v.tolist() == [7] and c.tolist() == [5]
    v, c = distinct([0, 1, 2, 3])
    assert v.tolist() == [0, 1, 2, 3] and c.tolist() == [1, 1, 1, 1]


def test_counts_partition_the_shots():
    rng = np.random.default_rng(0)
    x = rng.integers(0, 40, size=500)
    v, c = distinct(x)
    assert c.sum() == x.size and len(v) == len(set(x.tolist()))
    for val, cnt in zip(v.tolist(), c.tolist()):
        assert cnt == int(np.sum(x == val))
    firsts = [int(np.argmax(x == val)) for val in v.tolist()]
    assert firsts == sorted(firsts)


def test_expectation_limits_and_coupon_collector():
    p = np.full(16, 1 / 16)
    assert math.isclose(expected_distinct(p, 1), 1.0, rel_tol=1e-12)
    assert expected_distinct(p, 0) == 0.0
    assert math.isclose(expected_distinct([1.0, 0.0], 1000), 1.0, rel_tol=1e-12)
    assert math.isclose(expected_distinct(p, 10**6), 16.0, rel_tol=1e-12)
    # coupon collector: K (1 - (1 - 1/K)^m)
    assert math.isclose(expected_distinct(p, 20), 16 * (1 - (15 / 16) ** 20), rel_tol=1e-12)


def test_expectation_against_monte_carlo():
    rng = np.random.default_rng(3)
    p = rng.dirichlet(np.full(32, 0.5))
    m, trials = 25, 3000
    draws = rng.choice(32, size=(trials, m), p=p)
    counts = np.array([len(distinct(d)[0]) for d in draws], dtype=np.float64)
    mean, sd = counts.mean(), counts.std(ddof=1) / math.sqrt(trials)
    assert abs(mean - expected_distinct(p, m)) < 4.5 * sd


def test_sampler_shots_of_a_two_outcome_state():
    # |psi> on 1 qubit with p = (0.25, 0.75): 1000 shots have at most 2 distinct values
    psi = np.array([0.5, math.sqrt(0.75)], dtype=np.complex128)
    bits, _ = sample(psi, 1000, seed=1, cfg=0, alpha=0)
    v, c = distinct(bits)
    assert sorted(v.tolist()) == [0, 1] and c.sum() == 1000
    assert abs(c[v.tolist().index(1)] / 1000 - 0.75) < 5 * math.sqrt(0.75 * 0.25 / 1000)
