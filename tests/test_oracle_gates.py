"""Pins of the oracle's state-vector arithmetic against definitions and closed forms."""

import math

import numpy as np
import pytest

from oracle.gates import full_unitary, gate_matrix, kron_1q, u3, rot
from oracle.statevector import apply, zero_state


def _rand_unitary(rng, d):
    z = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _rand_state(rng, n):
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_apply_matches_bruteforce_operator(n):
    rng = np.random.default_rng(100 + n)
    for _ in range(6):
        k = int(rng.integers(1, min(n, 3) + 1))
        qs = tuple(int(q) for q in rng.choice(n, size=k, replace=False))
        U = _rand_unitary(rng, 1 << k)
        psi = _rand_state(rng, n)
        ref = full_unitary(n, U, qs) @ psi
        assert np.max(np.abs(apply(psi, n, U, qs) - ref)) < 1e-13


def test_kron_and_elementwise_builders_agree():
    rng = np.random.default_rng(7)
    for n in (1, 3, 5):
        for q in range(n):
            U = _rand_unitary(rng, 2)
            assert np.max(np.abs(kron_1q(n, U, q) - full_unitary(n, U, (q,)))) < 1e-15


def test_two_qubit_conventions_on_basis_states():
    n = 3
    # CNOT(control=0, target=2): |x0=1> -> |x0=1, x2=1>
    psi = np.zeros(8, dtype=complex); psi[1] = 1
    out = apply(psi, n, gate_matrix("CNOT"), (0, 2))
    assert out[5] == 1 and np.count_nonzero(out) == 1
    # control clear: nothing happens
    psi = np.zeros(8, dtype=complex); psi[4] = 1
    out = apply(psi, n, gate_matrix("CNOT"), (0, 2))
    assert out[4] == 1
    # CZ flips the sign of |11> only
    for x in range(8):
        psi = np.zeros(8, dtype=complex); psi[x] = 1
        out = apply(psi, n, gate_matrix("CZ"), (1, 2))
        assert out[x] == (-1 if (x >> 1) & 1 and (x >> 2) & 1 else 1)
    # SWAP exchanges the bits
    psi = np.zeros(8, dtype=complex); psi[2] = 1
    out = apply(psi, n, gate_matrix("SWAP"), (1, 2))
    assert out[4] == 1


def test_u3_textbook_special_cases():
    for th in (0.3, 1.7, 5.1):
        assert np.allclose(u3(th, 0.0, 0.0), rot("Y", th), atol=1e-15)
        assert np.allclose(u3(th, -math.pi / 2, math.pi / 2), rot("X", th), atol=1e-15)
    lam = 0.9
    # U3(0, 0, lam) = diag(1, e^{i lam}) = e^{i lam/2} RZ(lam)
    assert np.allclose(u3(0.0, 0.0, lam), np.exp(0.5j * lam) * rot("Z", lam), atol=1e-15)
    H = gate_matrix("H")
    assert np.allclose(u3(math.pi / 2, 0.0, math.pi), H, atol=1e-15)


def test_inverse_circuit_returns_to_zero():
    rng = np.random.default_rng(3)
    n = 6
    psi = zero_state(n)
    gates = []
    for _ in range(40):
        k = int(rng.integers(1, 3))
        qs = tuple(int(q) for q in rng.choice(n, size=k, replace=False))
        U = _rand_unitary(rng, 1 << k)
        gates.append((U, qs))
        psi = apply(psi, n, U, qs)
    for U, qs in reversed(gates):
        psi = apply(psi, n, U.conj().T, qs)
    assert abs(psi[0] - 1) < 1e-12 and np.max(np.abs(psi[1:])) < 1e-12


@pytest.mark.parametrize("n", [4, 9, 14])
def test_product_state_closed_form(n):
    rng = np.random.default_rng(n)
    angles = rng.uniform(0, 2 * math.pi, size=(n, 3))
    psi = zero_state(n)
    for q in range(n):
        psi = apply(psi, n, u3(*angles[q]), (q,))
    # <x| (x)_q U3_q |0> = prod_q (cos(t/2) if x_q = 0 else e^{i phi} sin(t/2))
    x = np.arange(1 << n)
    ref = np.ones(1 << n, dtype=complex)
    for q in range(n):
        t, ph, _ = angles[q]
        bit = (x >> q) & 1
        ref *= np.where(bit == 0, math.cos(t / 2), np.exp(1j * ph) * math.sin(t / 2))
    assert np.max(np.abs(psi - ref)) < 1e-13


@pytest.mark.parametrize("n", [2, 5, 12])
def test_ghz_closed_form(n):
    psi = apply(zero_state(n), n, gate_matrix("H"), (0,))
    for q in range(n - 1):
        psi = apply(psi, n, gate_matrix("CNOT"), (q, q + 1))
    ref = np.zeros(1 << n, dtype=complex)
    ref[0] = ref[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - ref)) < 1e-15


@pytest.mark.parametrize("n", [3, 7, 10])
def test_product_factors_equal_full_simulation(n):
    """product_factors / product_amplitudes against the full state vector for
    circuits of one-qubit gates, parameterised rotations and Pauli records."""
    from oracle.noise import expand
    from oracle.statevector import product_amplitudes, product_factors, run_record
    from workloads import product_circuit
    rng = np.random.default_rng(40 + n)
    circ = product_circuit(n, 3, rng, 0.1)
    circ["ops"].append({"kind": "param", "gen": "Y", "qubits": (n - 1,), "index": 0, "tag": "RY"})
    circ["params"] = [0.7]
    _, sites = expand(circ)
    rec = tuple(sorted((int(s), int(rng.integers(1, 4))) for s in rng.choice(len(sites), 4, replace=False)))
    psi, _ = run_record(circ, rec)
    f = product_factors(circ, rec)
    x = np.arange(1 << n)
    assert np.max(np.abs(product_amplitudes(f, x) - psi)) < 1e-13
    circ["ops"].append({"kind": "gate", "name": "CZ", "qubits": (0, 1), "params": (), "tag": "CZ"})
    with pytest.raises(ValueError):
        product_factors(circ, rec)
