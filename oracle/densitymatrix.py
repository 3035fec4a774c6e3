"""Exact density-matrix evolution for small circuits (Sec. 2.1: 2^n x 2^n).

rho <- G rho G^dagger for a gate; rho <- sum_k K_k rho K_k^dagger at a noise
site (pre-sampled or state-dependent alike); measure-reset on q is the channel {|0><0|, |0><1|} on q; PROJECT0 is
|0><0| followed by division by the trace.  Operators are lifted to the full
space with the brute-force builder of ``gates`` (n <= 8).
"""

import numpy as np

from .channels import kraus_ops
from .gates import full_unitary, gate_matrix, rot
from .noise import expand


def evolve(circuit, params=None):
    n = circuit["n_qubits"]
    N = 1 << n
    steps, sites = expand(circuit)
    if params is None:
        params = circuit.get("params", [])
    rho = np.zeros((N, N), dtype=np.complex128)
    rho[0, 0] = 1.0
    for st in steps:
        kind = st[0]
        if kind in ("gate", "param"):
            m = gate_matrix(st[1], st[3]) if kind == "gate" else rot(st[1], params[st[3]])
            U = full_unitary(n, m, st[2])
            rho = U @ rho @ U.conj().T
        elif kind == "site":
            ch = circuit["channels"][sites[st[1]]["channel"]]
            acc = np.zeros_like(rho)
            for K in kraus_ops(ch):
                F = full_unitary(n, K, st[2])
                acc += F @ rho @ F.conj().T
            rho = acc
        elif kind == "gch":
            acc = np.zeros_like(rho)
            for K in kraus_ops(circuit["channels"][st[3]]):
                F = full_unitary(n, K, st[1])
                acc += F @ rho @ F.conj().T
            rho = acc
        elif kind == "mr":
            acc = np.zeros_like(rho)
            for K in (np.array([[1, 0], [0, 0]], dtype=np.complex128),
                      np.array([[0, 1], [0, 0]], dtype=np.complex128)):
                F = full_unitary(n, K, st[1])
                acc += F @ rho @ F.conj().T
            rho = acc
        elif kind == "p0":
            F = full_unitary(n, np.array([[1, 0], [0, 0]], dtype=np.complex128), st[1])
            rho = F @ rho @ F.conj().T
            rho = rho / np.trace(rho).real
        else:
            raise ValueError(kind)
    return rho


def outcome_distribution(circuit, params=None):
    return np.real(np.diag(evolve(circuit, params))).copy()
