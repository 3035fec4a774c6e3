"""Conventional per-shot trajectories (Algorithm 1, Sec. 2.2).

Each shot re-prepares its own state: walk the operations in order, apply each
gate, and at every noise site draw r and apply U_k with k = index(r, {p_i})
(unitary-mixture branch, state-independent probabilities).  One shot is then
measured.  Shot i draws its site uniforms from word s of the stream
[seed, key1(BASELINE, cfg, i)] and its measurement uniform from the sampler
stream of trajectory i, so a PTS run with one shot per draw on the same streams
yields the same shots.
"""

import numpy as np

from .gates import gate_matrix, rot
from .noise import expand, site_channels
from .pts import _categorical
from .rng import key1, uniforms
from .sampling import sample
from .statevector import apply, zero_state

STREAM_BASELINE = 3


def per_shot(circuit, n_shots, seed, cfg, params=None):
    """Return (idx[n_shots], records) of ``n_shots`` conventional trajectories."""
    n = circuit["n_qubits"]
    steps, sites = expand(circuit)
    chans = site_channels(circuit)
    if params is None:
        params = circuit.get("params", [])
    out = np.zeros(n_shots, dtype=np.int64)
    recs = []
    for i in range(n_shots):
        r = uniforms(seed, key1(STREAM_BASELINE, cfg, i), len(sites)) if sites else []
        psi = zero_state(n)
        rec = []
        for st in steps:
            if st[0] == "gate":
                psi = apply(psi, n, gate_matrix(st[1], st[3]), st[2])
            elif st[0] == "param":
                psi = apply(psi, n, rot(st[1], params[st[3]]), st[2])
            elif st[0] == "site":
                probs, us = chans[sites[st[1]]["channel"]]
                k = _categorical(r[st[1]], probs)
                if k:
                    rec.append((st[1], k))
                psi = apply(psi, n, us[k], st[2])
            else:
                raise ValueError("per-shot baseline supports unitary operations only")
        idx, _ = sample(psi, 1, seed, cfg, i)
        out[i] = idx[0]
        recs.append(tuple(rec))
    return out, recs
