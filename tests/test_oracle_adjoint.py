"""Pins of the oracle's adjoint gradient: exact parameter shift and central differences."""

import numpy as np

from oracle.adjoint import ensemble_value, ensemble_value_and_grad, parameter_shift
from oracle.noise import site_probs
from oracle.pts import proportional
from workloads import random_small_circuit
from workloads.circuits import hea_circuit, zz_ring


def _setup(circ, T=24):
    sp = site_probs(circ)
    recs, counts = proportional(sp, 0, 5, T)
    w = [c / T for c in counts]
    return recs, w


def test_adjoint_matches_parameter_shift_hea():
    circ = hea_circuit(4, 2, np.random.default_rng(0), 0.08)
    recs, w = _setup(circ)
    terms = zz_ring(4)
    p = np.array(circ["params"])
    E, g = ensemble_value_and_grad(circ, recs, w, p, terms)
    ps = parameter_shift(circ, recs, w, p, terms)
    assert np.max(np.abs(g - ps)) < 1e-12
    assert abs(E - ensemble_value(circ, recs, w, p, terms)) < 1e-13


def test_adjoint_matches_central_difference_random_circuit():
    rng = np.random.default_rng(8)
    circ = random_small_circuit(4, 25, rng, with_params=True)
    assert len(circ["params"]) >= 3
    recs, w = _setup(circ, T=10)
    terms = [(0.7, (0, 1)), (-1.3, (2,)), (0.4, (1, 3))]
    p = np.array(circ["params"])
    _, g = ensemble_value_and_grad(circ, recs, w, p, terms)
    h = 1e-4
    for i in range(p.size):
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        fd = (ensemble_value(circ, recs, w, pp, terms) - ensemble_value(circ, recs, w, pm, terms)) / (2 * h)
        assert abs(fd - g[i]) < 1e-7
