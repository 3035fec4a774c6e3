"""Pins tying trajectories, PTS and the exact density-matrix channel together.

* Exhaustive identity: with every record of the product space and weight
  p_alpha, sum_alpha p_alpha |psi_alpha><psi_alpha| equals the exact density
  matrix (Fig. 2: the subsets' probabilities sum to one).
* Proportional PTS with multiplicity weights converges to rho at rate 1/sqrt(T).
* Most-likely-first truncation: TVD(truncated, exact) <= 1 - covered mass.
"""

import itertools
import math

import numpy as np

from oracle.densitymatrix import evolve
from oracle.noise import expand, site_channels, site_probs
from oracle.pts import joint_prob, most_likely, proportional
from oracle.statevector import run_record
from workloads import random_small_circuit


def _all_records(sp):
    for ks in itertools.product(*[range(len(p)) for p in sp]):
        yield tuple((s, k) for s, k in enumerate(ks) if k)


def _tiny_circuit(seed, n=3, gates=7):
    rng = np.random.default_rng(seed)
    return random_small_circuit(n, gates, rng, p1=0.15, p2=0.2)


def test_exhaustive_records_reproduce_density_matrix():
    for seed in range(4):
        circ = _tiny_circuit(seed)
        sp = site_probs(circ)
        if int(np.prod([len(p) for p in sp])) > 40000:
            continue
        ss = expand(circ)
        ch = site_channels(circ)
        rho = evolve(circ)
        acc = np.zeros_like(rho)
        total = 0.0
        for rec in _all_records(sp):
            psi, _ = run_record(circ, rec, steps_sites=ss, chans=ch)
            pa = joint_prob(rec, sp)
            acc += pa * np.outer(psi, psi.conj())
            total += pa
        assert abs(total - 1.0) < 1e-12
        assert np.max(np.abs(acc - rho)) < 1e-12


def test_proportional_ensemble_converges_as_inverse_sqrt_T():
    circ = random_small_circuit(3, 12, np.random.default_rng(21), p1=0.3, p2=0.4)
    sp = site_probs(circ)
    ss = expand(circ)
    ch = site_channels(circ)
    rho = evolve(circ)
    Ts = [2 ** k for k in range(6, 12)]
    errs = []
    for T in Ts:
        e2 = []
        for rep in range(4):
            recs, counts = proportional(sp, 100 + rep, 1, T)
            acc = np.zeros_like(rho)
            for rec, c in zip(recs, counts):
                psi, _ = run_record(circ, rec, steps_sites=ss, chans=ch)
                acc += (c / T) * np.outer(psi, psi.conj())
            e2.append(np.linalg.norm(acc - rho) ** 2)
        errs.append(math.sqrt(np.mean(e2)))
    slope = np.polyfit(np.log(Ts), np.log(errs), 1)[0]
    assert -0.65 < slope < -0.35, slope


def test_most_likely_truncation_bound():
    circ = random_small_circuit(3, 10, np.random.default_rng(4), p1=0.05, p2=0.1)
    sp = site_probs(circ)
    ss = expand(circ)
    ch = site_channels(circ)
    exact = np.real(np.diag(evolve(circ)))
    for K in (1, 4, 30):
        recs, _ = most_likely(sp, K)
        ps = [joint_prob(r, sp) for r in recs]
        cover = math.fsum(ps)
        dist = np.zeros_like(exact)
        for rec, pa in zip(recs, ps):
            psi, _ = run_record(circ, rec, steps_sites=ss, chans=ch)
            dist += (pa / cover) * np.abs(psi) ** 2
        tvd = 0.5 * np.sum(np.abs(dist - exact))
        assert tvd <= (1 - cover) + 1e-12


def test_ensemble_weights_reproduce_the_channel_expectation():
    """sample_kraus's weights: most-likely-first over every record with reweight
    weights (p_alpha / sum p) gives Tr(O rho) of the exact channel; with
    multiplicity weights they are the draw frequencies count / T; uniform
    weights are equal.  O = Z_0 Z_1 + 0.5 Z_2 (diagonal)."""
    from oracle.pts import ensemble_weights, sample_kraus
    circ = _tiny_circuit(1)
    sp = site_probs(circ)
    n_all = int(np.prod([len(p) for p in sp]))
    ss = expand(circ)
    ch = site_channels(circ)
    rho = evolve(circ)
    x = np.arange(1 << circ["n_qubits"])
    z = lambda q: 1 - 2 * ((x >> q) & 1)
    odiag = z(0) * z(1) + 0.5 * z(2)
    exact = float(np.real(np.sum(np.diag(rho) * odiag)))
    ref = sample_kraus(sp, {"mode": "most_likely", "k_max": n_all, "total_shots": 10 ** 6,
                            "alloc": "reweight"}, 0, 1)
    assert len(ref["records"]) == n_all
    e = 0.0
    for rec, w in zip(ref["records"], ref["weights"]):
        psi, _ = run_record(circ, rec, steps_sites=ss, chans=ch)
        e += w * float(np.sum(np.abs(psi) ** 2 * odiag))
    assert abs(e - exact) < 1e-12
    ref = sample_kraus(sp, {"mode": "proportional", "n_draws": 500, "total_shots": 999,
                            "alloc": "multiplicity"}, 3, 1)
    assert np.allclose(ref["weights"], np.asarray(ref["counts"]) / 500.0, rtol=0, atol=1e-15)
    assert ensemble_weights([5, 1, 2], [0.1, 0.2, 0.3], "uniform") == [1 / 3] * 3
