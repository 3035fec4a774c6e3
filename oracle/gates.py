"""Gate matrices (complex128) and a brute-force full-unitary builder.

Convention: basis index x = sum_q x_q 2^q.  A k-qubit gate on qubits
(q_0, ..., q_{k-1}) has matrix row/column bit j <-> qubit q_j, so bit 0 of the
matrix index is q_0.  The paper fixes no convention (Sec. 2.1 only defines the
2^n vector); this is the reading used throughout.
"""

import math

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULIS = (I2, X, Y, Z)


def u3(theta, phi, lam):
    c = math.cos(theta / 2.0)
    s = math.sin(theta / 2.0)
    return np.array([[c, -np.exp(1j * lam) * s],
                     [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]], dtype=np.complex128)


def rot(gen, theta):
    """exp(-i theta P / 2) for P in {X, Y, Z}."""
    P = {"X": X, "Y": Y, "Z": Z}[gen]
    return math.cos(theta / 2.0) * I2 - 1j * math.sin(theta / 2.0) * P


def rot_derivative(gen, theta):
    """d/dtheta exp(-i theta P/2) = (-i/2) P exp(-i theta P/2)."""
    P = {"X": X, "Y": Y, "Z": Z}[gen]
    return (-0.5j) * P @ rot(gen, theta)


def gate_matrix(name, params=()):
    if name == "U3":
        return u3(*params)
    if name in ("RX", "RY", "RZ"):
        return rot(name[1], params[0])
    if name == "H":
        return np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
    if name == "X":
        return X.copy()
    if name == "Y":
        return Y.copy()
    if name == "Z":
        return Z.copy()
    if name == "S":
        return np.diag([1, 1j]).astype(np.complex128)
    if name == "T":
        return np.diag([1, np.exp(1j * math.pi / 4)]).astype(np.complex128)
    if name == "CZ":
        return np.diag([1, 1, 1, -1]).astype(np.complex128)
    if name == "CNOT":
        # qubits = (control, target); index = c + 2 t
        m = np.zeros((4, 4), dtype=np.complex128)
        for c in (0, 1):
            for t in (0, 1):
                m[c + 2 * (t ^ c), c + 2 * t] = 1.0
        return m
    if name == "SWAP":
        m = np.zeros((4, 4), dtype=np.complex128)
        for a in (0, 1):
            for b in (0, 1):
                m[b + 2 * a, a + 2 * b] = 1.0
        return m
    raise ValueError(f"unknown gate {name}")


def full_unitary(n, mat, qubits):
    """Brute-force 2^n x 2^n operator of a k-qubit matrix on ``qubits``.

    Entry [y, x] = mat[r(y), c(x)] when y and x agree on every non-target bit,
    else 0, with r, c the matrix indices built from the target bits.  Written
    straight from the definition, element by element (n <= 6).
    """
    N = 1 << n
    k = len(qubits)
    out = np.zeros((N, N), dtype=np.complex128)
    tmask = 0
    for q in qubits:
        tmask |= 1 << q
    for x in range(N):
        cx = sum(((x >> q) & 1) << j for j, q in enumerate(qubits))
        for r in range(1 << k):
            y = x & ~tmask
            for j, q in enumerate(qubits):
                y |= ((r >> j) & 1) << q
            out[y, x] = mat[r, cx]
    return out


def kron_1q(n, mat, q):
    """Full operator of a 1-qubit matrix via Kronecker products, highest qubit first."""
    out = np.array([[1.0 + 0j]])
    for qq in range(n - 1, -1, -1):
        out = np.kron(out, mat if qq == q else I2)
    return out
