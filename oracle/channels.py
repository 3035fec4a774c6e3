"""Kraus channels, the CPTP condition and unitary-mixture detection.

Sec. 2.2 (noise-channel paragraph): a channel is a set of Kraus operators
{K_i} with sum_i K_i^dagger K_i = I (CPTP); a trajectory applies K_i with
probability <psi|K_i^dagger K_i|psi>.  Feature 2 of the same section: a
unitary-mixture channel has K_i proportional to a unitary U_i.  The printed
"K_i = p_i U_i" is read as K_i = sqrt(p_i) U_i, i.e. K_i^dagger K_i = p_i I,
which makes p_i independent of the state.

Conventions (the paper names none):
* depolarizing(1q, p): {sqrt(1-p) I, sqrt(p/3) X, sqrt(p/3) Y, sqrt(p/3) Z};
* depolarizing(2q, p): {sqrt(1-p) II} then sqrt(p/15) P_a (x) P_b for the 15
  non-identity pairs, index k = 4a + b in I,X,Y,Z order, where P_a acts on the
  site's second qubit (matrix bit 1) and P_b on its first (matrix bit 0);
* xflip(p): {sqrt(1-p) I, sqrt(p) X};
* pauli(px, py, pz): {sqrt(1-px-py-pz) I, sqrt(px) X, sqrt(py) Y, sqrt(pz) Z};
* u3_mixture(p, angles): {sqrt(1-p) I, sqrt(p) U3(angles)};
* amplitude_damping(gamma): {[[1,0],[0,sqrt(1-gamma)]], [[0,sqrt(gamma)],[0,0]]}.
Index 0 is the no-error operator of every channel above.  A channel may also be
given as {"kraus": [K_0, K_1, ...]}.

Pauli twirl (Sec. 1 names Pauli-twirled noise among the tailored error
models): averaging E over rho -> P^dag E(P rho P^dag) P for every Pauli string P
leaves a Pauli channel whose probabilities are p_P = sum_k |Tr(P^dag K_k)|^2 /
d^2.  Strings are indexed by base-4 digits (0 I, 1 X, 2 Y, 3 Z), digit j on the
site's qubit j (matrix bit j, the least significant factor of np.kron).
"""

import math

import numpy as np

from .gates import PAULIS, u3, I2


def kraus_ops(ch):
    if "kraus" in ch:
        return [np.asarray(k, dtype=np.complex128) for k in ch["kraus"]]
    name = ch["name"]
    if name == "depolarizing":
        p = ch["p"]
        if ch["nq"] == 1:
            a0 = math.sqrt(1.0 - p)
            a = math.sqrt(p / 3.0)
            return [a0 * PAULIS[0]] + [a * P for P in PAULIS[1:]]
        a0 = math.sqrt(1.0 - p)
        a = math.sqrt(p / 15.0)
        ops = []
        for ia in range(4):
            for ib in range(4):
                m = np.kron(PAULIS[ia], PAULIS[ib])
                ops.append((a0 if (ia == 0 and ib == 0) else a) * m)
        return ops
    if name == "xflip":
        p = ch["p"]
        return [math.sqrt(1.0 - p) * PAULIS[0], math.sqrt(p) * PAULIS[1]]
    if name == "pauli":
        px, py, pz = ch["probs"]
        return [math.sqrt(1.0 - px - py - pz) * PAULIS[0], math.sqrt(px) * PAULIS[1],
                math.sqrt(py) * PAULIS[2], math.sqrt(pz) * PAULIS[3]]
    if name == "u3_mixture":
        p = ch["p"]
        return [math.sqrt(1.0 - p) * I2, math.sqrt(p) * u3(*ch["params"])]
    if name == "amplitude_damping":
        g = ch["gamma"]
        return [np.array([[1, 0], [0, math.sqrt(1.0 - g)]], dtype=np.complex128),
                np.array([[0, math.sqrt(g)], [0, 0]], dtype=np.complex128)]
    raise ValueError(f"unknown channel {name}")


def cptp_error(kraus):
    """max_ij | (sum_k K_k^dagger K_k - I)_ij |."""
    d = kraus[0].shape[0]
    acc = np.zeros((d, d), dtype=np.complex128)
    for K in kraus:
        acc += K.conj().T @ K
    return float(np.max(np.abs(acc - np.eye(d))))


def kraus_weight(K):
    """tr(K^dagger K) / d, summed element by element in row-major order.

    For K = sqrt(p) U this is p.  A plain sequential loop, so the value does not
    depend on a library's summation order."""
    d = K.shape[0]
    s = 0.0
    for i in range(d):
        for j in range(d):
            z = K[i, j]
            s += z.real * z.real + z.imag * z.imag
    return s / d


def unitary_mixture(kraus, tol=1e-12):
    """Return (probs, unitaries) if every K_k^dagger K_k = p_k I within ``tol``, else None.

    U_k = K_k / sqrt(p_k); a zero-probability operator keeps U_k = I (never drawn)."""
    d = kraus[0].shape[0]
    probs = []
    unitaries = []
    for K in kraus:
        p = kraus_weight(K)
        if np.max(np.abs(K.conj().T @ K - p * np.eye(d))) > tol:
            return None
        probs.append(p)
        unitaries.append(K / math.sqrt(p) if p > 0 else np.eye(d, dtype=np.complex128))
    return probs, unitaries


def pauli_string(index, nq):
    """The Pauli string with base-4 digit j (0 I, 1 X, 2 Y, 3 Z) on matrix bit j."""
    m = np.ones((1, 1), dtype=np.complex128)
    for j in reversed(range(nq)):
        m = np.kron(m, PAULIS[(index >> (2 * j)) & 3])
    return m


def pauli_twirl(kraus):
    """p_P = sum_k |Tr(P^dag K_k)|^2 / d^2 for every Pauli string P (the definition)."""
    d = kraus[0].shape[0]
    nq = d.bit_length() - 1
    out = np.zeros(4 ** nq)
    for i in range(4 ** nq):
        P = pauli_string(i, nq)
        out[i] = sum(abs(np.trace(P.conj().T @ K)) ** 2 for K in kraus) / d ** 2
    return out


def twirled(ch):
    """The channel dict of ch's Pauli twirl: sqrt(p_P) P for p_P > 0, in string order."""
    K = kraus_ops(ch)
    nq = K[0].shape[0].bit_length() - 1
    p = pauli_twirl(K)
    return {"kraus": [math.sqrt(p[i]) * pauli_string(i, nq) for i in range(p.size) if p[i] > 0],
            "nq": nq}


def pauli_transfer_diagonal(kraus):
    """R_PP = Tr(P^dag E(P)) / d for every Pauli string P."""
    d = kraus[0].shape[0]
    nq = d.bit_length() - 1
    out = np.zeros(4 ** nq)
    for i in range(4 ** nq):
        P = pauli_string(i, nq)
        EP = sum(K @ P @ K.conj().T for K in kraus)
        out[i] = np.trace(P.conj().T @ EP).real / d
    return out


def state_dependent(kraus, tol=1e-12):
    """A CPTP channel on one or two qubits that is not a unitary mixture: its
    probabilities p_k = <psi|K_k^dagger K_k|psi> depend on the state, so it is
    resolved when the trajectory's state reaches it (Algorithm 1's
    state-dependent branch) instead of being pre-sampled."""
    return kraus[0].shape in ((2, 2), (4, 4)) and unitary_mixture(kraus, tol) is None


def general_channel(kraus, tol=1e-12):
    """A state-dependent channel on one qubit with every K_k^dagger K_k diagonal
    (amplitude damping, phase damping) has p_k = d0[k] P(q=0) + d1[k] P(q=1), a
    function of the qubit's populations alone.  Returns (d0, d1), or None for
    any other channel."""
    if unitary_mixture(kraus, tol) is not None or kraus[0].shape != (2, 2):
        return None
    d0, d1 = [], []
    for K in kraus:
        m = K.conj().T @ K
        if abs(m[0, 1]) > tol or abs(m[1, 0]) > tol:
            return None
        d0.append(float(m[0, 0].real))
        d1.append(float(m[1, 1].real))
    return d0, d1
