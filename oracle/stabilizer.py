"""Pauli-frame propagation (Gottesman-Knill) for Clifford circuits with Pauli noise.

Used only to pin the measure-reset records of the surface-code workload: the
noiseless circuit after its projection round reports every stabiliser as +1
(outcome 0), so a trajectory's outcome at a measure-reset is the X component of
its Pauli frame on that ancilla.  Rules: H swaps the X and Z components;
CNOT(c, t) does x_t ^= x_c and z_c ^= z_t; a Pauli error XORs its components;
measure-reset and PROJECT0 clear the qubit's frame.
"""

import numpy as np

from .gates import PAULIS
from .noise import expand, site_channels


def _pauli_label(U):
    """Return (x bits, z bits) of a 1- or 2-qubit Pauli operator (up to phase)."""
    d = U.shape[0]
    if d == 2:
        for i, P in enumerate(PAULIS):
            ov = np.vdot(P, U)
            if abs(abs(ov) - 2.0) < 1e-9:
                return [i in (1, 2)], [i in (2, 3)]
    else:
        for a in range(4):
            for b in range(4):
                P = np.kron(PAULIS[a], PAULIS[b])
                ov = np.vdot(P, U)
                if abs(abs(ov) - 4.0) < 1e-9:
                    # matrix bit 0 <-> first qubit (P_b), bit 1 <-> second qubit (P_a)
                    return [b in (1, 2), a in (1, 2)], [b in (2, 3), a in (2, 3)]
    raise ValueError("not a Pauli operator")


def frame_run(circuit, record):
    """Return (mr_bits, final x-frame as an int bitmask) for one record."""
    n = circuit["n_qubits"]
    steps, sites = expand(circuit)
    chans = site_channels(circuit)
    ks = dict(record)
    x = [False] * n
    z = [False] * n
    bits = []
    for st in steps:
        kind = st[0]
        if kind == "gate":
            name, qs = st[1], st[2]
            if name == "H":
                q = qs[0]
                x[q], z[q] = z[q], x[q]
            elif name == "CNOT":
                c, t = qs
                x[t] ^= x[c]
                z[c] ^= z[t]
            else:
                raise ValueError(f"frame propagation does not support {name}")
        elif kind == "site":
            k = ks.get(st[1], 0)
            if k == 0:
                continue
            _, us = chans[sites[st[1]]["channel"]]
            xs, zs = _pauli_label(us[k])
            for j, q in enumerate(st[2]):
                x[q] ^= xs[j]
                z[q] ^= zs[j]
        elif kind == "mr":
            q = st[1][0]
            bits.append(1 if x[q] else 0)
            x[q] = z[q] = False
        elif kind == "p0":
            q = st[1][0]
            x[q] = z[q] = False
        else:
            raise ValueError(kind)
    mask = 0
    for q in range(n):
        if x[q]:
            mask |= 1 << q
    return bits, mask
