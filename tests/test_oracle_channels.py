"""Pins of the oracle's channels: CPTP, unitary-mixture probabilities, textbook
channel actions, and the unnormalised-Kraus norm invariant ||psi_alpha||^2 = p_alpha."""

import math

import numpy as np
import pytest

from oracle.channels import cptp_error, kraus_ops, unitary_mixture
from oracle.gates import PAULIS
from oracle.noise import expand, site_probs
from oracle.pts import joint_prob, proportional
from oracle.statevector import run_record
from workloads import random_small_circuit

CHANNELS = [
    {"name": "depolarizing", "nq": 1, "p": 0.013},
    {"name": "depolarizing", "nq": 2, "p": 0.021},
    {"name": "xflip", "nq": 1, "p": 0.2},
    {"name": "pauli", "nq": 1, "probs": (0.03, 0.02, 0.05)},
    {"name": "u3_mixture", "nq": 1, "p": 0.07, "params": (0.4, 1.1, 2.9)},
    {"name": "amplitude_damping", "nq": 1, "gamma": 0.3},
]


@pytest.mark.parametrize("ch", CHANNELS, ids=lambda c: c["name"] + str(c.get("nq", 1)))
def test_cptp(ch):
    assert cptp_error(kraus_ops(ch)) < 1e-12


def test_unitary_mixture_probabilities_closed_form():
    p = 0.013
    probs, us = unitary_mixture(kraus_ops(CHANNELS[0]))
    assert np.allclose(probs, [1 - p, p / 3, p / 3, p / 3], rtol=1e-14, atol=0)
    probs, _ = unitary_mixture(kraus_ops(CHANNELS[1]))
    assert len(probs) == 16
    assert np.allclose(probs, [1 - 0.021] + [0.021 / 15] * 15, rtol=1e-14, atol=0)
    probs, _ = unitary_mixture(kraus_ops(CHANNELS[3]))
    assert np.allclose(probs, [0.9, 0.03, 0.02, 0.05], rtol=1e-14, atol=0)
    for u in us:
        assert np.allclose(u.conj().T @ u, np.eye(2), atol=1e-14)
    assert unitary_mixture(kraus_ops(CHANNELS[5])) is None


def _rand_rho(rng, d):
    a = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    r = a @ a.conj().T
    return r / np.trace(r)


def test_depolarizing_textbook_action():
    """rho -> (1 - 4p/3) rho + (4p/3) I/2 (1q) and (1 - 16p/15) rho + (16p/15) I/4 (2q)."""
    rng = np.random.default_rng(1)
    for ch, d, f in ((CHANNELS[0], 2, 4.0 / 3.0), (CHANNELS[1], 4, 16.0 / 15.0)):
        rho = _rand_rho(rng, d)
        out = sum(K @ rho @ K.conj().T for K in kraus_ops(ch))
        ref = (1 - f * ch["p"]) * rho + f * ch["p"] * np.eye(d) / d
        assert np.max(np.abs(out - ref)) < 1e-15


def test_two_qubit_pauli_order():
    """k = 4a + b: P_a on the site's second qubit (matrix bit 1), P_b on its first."""
    K = kraus_ops(CHANNELS[1])
    a, b = 1, 3   # X on the second qubit, Z on the first
    U = K[4 * a + b] / math.sqrt(0.021 / 15)
    assert np.allclose(U, np.kron(PAULIS[1], PAULIS[3]))
    # acting on |x0=0, x1=0>: Z on bit 0 gives +1, X on bit 1 moves to index 2
    v = U @ np.array([1, 0, 0, 0], dtype=complex)
    assert np.allclose(v, [0, 0, 1, 0])


def test_unnormalised_kraus_norm_is_joint_probability():
    rng = np.random.default_rng(11)
    circ = random_small_circuit(4, 30, rng, p1=0.2, p2=0.3)
    probs = site_probs(circ)
    recs, _ = proportional(probs, 0, 9, 40)
    for rec in recs:
        psi, _ = run_record(circ, rec, kraus_unnormalised=True)
        nrm = math.fsum(psi.real ** 2 + psi.imag ** 2)
        assert abs(nrm - joint_prob(rec, probs)) <= 1e-12 * joint_prob(rec, probs)


def test_site_expansion_order_rules():
    circ = {"n_qubits": 2,
            "ops": [{"kind": "gate", "name": "H", "qubits": (0,), "params": (), "tag": "H"},
                    {"kind": "gate", "name": "CZ", "qubits": (0, 1), "params": (), "tag": "CZ"},
                    {"kind": "measure_reset", "qubits": (1,)},
                    {"kind": "noise", "channel": 0, "qubits": (1,)}],
            "channels": [{"name": "xflip", "nq": 1, "p": 0.1},
                         {"name": "depolarizing", "nq": 2, "p": 0.1}],
            "rules": [{"when": "after_tag", "tag": "H", "channel": 0},
                      {"when": "after_tag", "tag": "CZ", "channel": 1},
                      {"when": "before_measure", "channel": 0},
                      {"when": "before_readout", "qubits": (1, 0), "channel": 0}]}
    steps, sites = expand(circ)
    kinds = [s[0] for s in steps]
    assert kinds == ["gate", "site", "gate", "site", "site", "mr", "site", "site", "site"]
    assert [s["qubits"] for s in sites] == [(0,), (0, 1), (1,), (1,), (0,), (1,)]


# ---------------------------------------------------------------- Pauli twirl

def _random_cptp(nq, n_kraus, rng):
    d = 2 ** nq
    a = rng.normal(size=(n_kraus * d, d)) + 1j * rng.normal(size=(n_kraus * d, d))
    q, _ = np.linalg.qr(a)                                 # isometry: sum K^dag K = I
    return [q[k * d:(k + 1) * d, :] for k in range(n_kraus)]


def test_twirl_of_amplitude_damping_closed_form():
    from oracle.channels import pauli_twirl
    for g in (0.0, 0.1, 0.37, 1.0):
        s = math.sqrt(1 - g)
        p = pauli_twirl(kraus_ops({"name": "amplitude_damping", "gamma": g}))
        assert np.allclose(p, [(1 + s) ** 2 / 4, g / 4, g / 4, (1 - s) ** 2 / 4], atol=1e-15)


def test_twirl_fixed_points_and_unitaries():
    from oracle.channels import pauli_twirl
    p = pauli_twirl(kraus_ops({"name": "pauli", "probs": (0.03, 0.02, 0.05)}))
    assert np.allclose(p, [0.9, 0.03, 0.02, 0.05], atol=1e-15)
    p = pauli_twirl(kraus_ops({"name": "depolarizing", "nq": 2, "p": 0.3}))
    assert np.allclose(p, [0.7] + [0.02] * 15, atol=1e-15)
    th = 0.8
    rz = np.diag([np.exp(-0.5j * th), np.exp(0.5j * th)])
    assert np.allclose(pauli_twirl([rz]), [math.cos(th / 2) ** 2, 0, 0, math.sin(th / 2) ** 2], atol=1e-15)


def test_twirl_keeps_the_transfer_diagonal_and_sums_to_one():
    from oracle.channels import pauli_transfer_diagonal, pauli_twirl, twirled
    rng = np.random.default_rng(9)
    for nq, nk in ((1, 2), (1, 3), (2, 2), (2, 5)):
        K = _random_cptp(nq, nk, rng)
        p = pauli_twirl(K)
        assert abs(p.sum() - 1) < 1e-12 and np.all(p >= 0)
        Kt = twirled({"kraus": K})["kraus"]
        assert np.allclose(pauli_transfer_diagonal(K), pauli_transfer_diagonal(Kt), atol=1e-12)


def test_twirl_string_index_puts_digit_j_on_matrix_bit_j():
    from oracle.channels import pauli_twirl
    ad = kraus_ops({"name": "amplitude_damping", "gamma": 0.5})
    on_bit0 = [np.kron(np.eye(2), A) for A in ad]          # acts on the site's first qubit only
    p = pauli_twirl(on_bit0)
    assert np.all(p.reshape(4, 4)[1:, :] == 0)             # digit 1 (second qubit) is always I
    assert np.allclose(p[:4], pauli_twirl(ad), atol=1e-15)
