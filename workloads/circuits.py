"""Symbolic, seeded circuit and noise-model generators.

Everything here is a plain description: gate names with angles, channel names
with probabilities, and sampling options.  Both the oracle and the GPU path turn
these descriptions into matrices with their own code.

Circuit dictionary layout::

    {"n_qubits": n,
     "ops": [ {"kind": "gate", "name": "U3", "qubits": (q,), "params": (t, p, l), "tag": "U3"},
              {"kind": "param", "gen": "Y", "qubits": (q,), "index": i, "tag": "RY"},
              {"kind": "noise", "channel": c, "qubits": (a, b)},
              {"kind": "measure_reset", "qubits": (q,)},
              {"kind": "project0", "qubits": (q,)} ],
     "channels": [ {"name": "depolarizing", "nq": 1, "p": 1e-3}, ... ],
     "rules": [ {"when": "after_tag", "tag": "U3", "channel": 0},
                {"when": "before_measure", "channel": 2},
                {"when": "before_readout", "qubits": (0, 1), "channel": 2} ],
     "params": [...]}          # values of the "param" ops, if any

Gate names: U3(theta, phi, lambda), RX, RY, RZ (one angle), H, X, Y, Z, S, T,
CZ, CNOT (qubits = (control, target)), SWAP.
Channel names: depolarizing (nq 1 or 2, p), xflip (p), pauli (probs = [px, py, pz]),
u3_mixture (p, params = U3 angles: K0 = sqrt(1-p) I, K1 = sqrt(p) U3),
amplitude_damping (gamma; not a unitary mixture).
"""

import math

import numpy as np

# Counter-RNG stream identifiers.  Every random draw of the method is taken from
# a Philox4x64-10 stream keyed [seed, key1(stream, cfg, i)].
STREAM_PTS = 1
STREAM_SAMPLER = 2
STREAM_BASELINE = 3


def key1(stream, cfg, i):
    """Second key word of a Philox stream: stream id, workload id and item index."""
    return (int(stream) << 56) | (int(cfg) << 48) | int(i)


def _brick_pairs(n, layer):
    start = layer % 2
    return [(a, a + 1) for a in range(start, n - 1, 2)]


def brick_circuit(n, layers, rng, p1, p2, eps_sigma=None, explicit_noise=False):
    """Random U3 on every qubit, then CZ on alternating brick pairs (open boundary).

    Layer l uses pairs (0,1),(2,3),... when l is even and (1,2),(3,4),... when odd.
    With ``eps_sigma`` a fixed coherent over-rotation RZ(eps) is applied to both
    qubits of each CZ right after it, eps ~ N(0, eps_sigma^2), one draw per CZ.
    Noise: 1-qubit depolarizing p1 after each U3 and 2-qubit depolarizing p2
    after each CZ (after its over-rotation), either as tag rules or as explicit
    noise ops.
    """
    ops = []
    channels = []
    rules = []
    ch1 = ch2 = None
    if p1 > 0:
        ch1 = len(channels)
        channels.append({"name": "depolarizing", "nq": 1, "p": float(p1)})
    if p2 > 0:
        ch2 = len(channels)
        channels.append({"name": "depolarizing", "nq": 2, "p": float(p2)})
    use_explicit = explicit_noise or eps_sigma is not None
    if not use_explicit:
        if ch1 is not None:
            rules.append({"when": "after_tag", "tag": "U3", "channel": ch1})
        if ch2 is not None:
            rules.append({"when": "after_tag", "tag": "CZ", "channel": ch2})
    for layer in range(layers):
        angles = rng.uniform(0.0, 2.0 * math.pi, size=(n, 3))
        pairs = _brick_pairs(n, layer)
        eps = rng.normal(0.0, eps_sigma, size=len(pairs)) if eps_sigma is not None else None
        for q in range(n):
            ops.append({"kind": "gate", "name": "U3", "qubits": (q,),
                        "params": tuple(float(a) for a in angles[q]), "tag": "U3"})
            if use_explicit and ch1 is not None:
                ops.append({"kind": "noise", "channel": ch1, "qubits": (q,)})
        for j, (a, b) in enumerate(pairs):
            ops.append({"kind": "gate", "name": "CZ", "qubits": (a, b), "params": (), "tag": "CZ"})
            if eps is not None:
                e = float(eps[j])
                ops.append({"kind": "gate", "name": "RZ", "qubits": (a,), "params": (e,), "tag": "RZ"})
                ops.append({"kind": "gate", "name": "RZ", "qubits": (b,), "params": (e,), "tag": "RZ"})
            if use_explicit and ch2 is not None:
                ops.append({"kind": "noise", "channel": ch2, "qubits": (a, b)})
    return {"n_qubits": n, "ops": ops, "channels": channels, "rules": rules, "params": []}


# Rotated distance-3 surface code: data qubits 0..8 on a 3x3 grid (index 3r+c),
# ancillas 9..16.  Bulk faces (i, j) cover data (i,j),(i,j+1),(i+1,j),(i+1,j+1)
# and alternate X/Z in a checkerboard; X-type weight-2 faces sit on the top and
# bottom edges, Z-type weight-2 faces on the left and right edges.
SURFACE_D3_CHECKS = (
    ("X", (0, 1, 3, 4)),   # ancilla 9
    ("Z", (1, 2, 4, 5)),   # ancilla 10
    ("Z", (3, 4, 6, 7)),   # ancilla 11
    ("X", (4, 5, 7, 8)),   # ancilla 12
    ("X", (1, 2)),         # ancilla 13, top edge
    ("X", (6, 7)),         # ancilla 14, bottom edge
    ("Z", (0, 3)),         # ancilla 15, left edge
    ("Z", (5, 8)),         # ancilla 16, right edge
)


def surface_code_d3(rounds=5, p=1e-3, p_meas=1e-3, projection_round=True):
    """Memory experiment on the rotated d=3 surface code (9 data + 8 ancilla qubits).

    A noiseless projection round (extraction circuit, then PROJECT0 on each
    ancilla) prepares the logical |0>.  Each of the ``rounds`` noisy rounds runs
    the extraction circuit (Z-check: CNOT data->ancilla; X-check: H, CNOT
    ancilla->data, H) and then a mid-circuit measure-reset of every ancilla.
    Noise: 1-qubit depolarizing p after every noisy H, 2-qubit depolarizing p
    after every noisy CNOT, an X-flip p_meas before every measure-reset and
    before the final readout of each data qubit.
    """
    n = 17
    ops = []

    def extraction(noisy):
        h, cx = ("H", "CNOT") if noisy else ("H0", "CNOT0")
        for a, (kind, support) in enumerate(SURFACE_D3_CHECKS):
            anc = 9 + a
            if kind == "Z":
                for d in support:
                    ops.append({"kind": "gate", "name": "CNOT", "qubits": (d, anc), "params": (), "tag": cx})
            else:
                ops.append({"kind": "gate", "name": "H", "qubits": (anc,), "params": (), "tag": h})
                for d in support:
                    ops.append({"kind": "gate", "name": "CNOT", "qubits": (anc, d), "params": (), "tag": cx})
                ops.append({"kind": "gate", "name": "H", "qubits": (anc,), "params": (), "tag": h})

    if projection_round:
        extraction(False)
        for a in range(8):
            ops.append({"kind": "project0", "qubits": (9 + a,)})
    for _ in range(rounds):
        extraction(True)
        for a in range(8):
            ops.append({"kind": "measure_reset", "qubits": (9 + a,)})
    channels = [
        {"name": "depolarizing", "nq": 1, "p": float(p)},
        {"name": "depolarizing", "nq": 2, "p": float(p)},
        {"name": "xflip", "nq": 1, "p": float(p_meas)},
    ]
    rules = [
        {"when": "after_tag", "tag": "H", "channel": 0},
        {"when": "after_tag", "tag": "CNOT", "channel": 1},
        {"when": "before_measure", "channel": 2},
        {"when": "before_readout", "qubits": tuple(range(9)), "channel": 2},
    ]
    return {"n_qubits": n, "ops": ops, "channels": channels, "rules": rules, "params": []}


def hea_circuit(n, layers, rng, p2):
    """Hardware-efficient ansatz: per layer RY(theta_q) RZ(phi_q) on every qubit,
    then CZ(i, i+1 mod n) for i = 0..n-1, each followed by 2-qubit depolarizing p2.
    Parameter index of RY on qubit q in layer l is l*2n + 2q, of RZ that plus one.
    """
    ops = []
    for layer in range(layers):
        for q in range(n):
            base = layer * 2 * n + 2 * q
            ops.append({"kind": "param", "gen": "Y", "qubits": (q,), "index": base, "tag": "RY"})
            ops.append({"kind": "param", "gen": "Z", "qubits": (q,), "index": base + 1, "tag": "RZ"})
        for i in range(n):
            ops.append({"kind": "gate", "name": "CZ", "qubits": (i, (i + 1) % n), "params": (), "tag": "CZ"})
    params = rng.uniform(0.0, 2.0 * math.pi, size=layers * 2 * n)
    channels = [{"name": "depolarizing", "nq": 2, "p": float(p2)}]
    rules = [{"when": "after_tag", "tag": "CZ", "channel": 0}]
    return {"n_qubits": n, "ops": ops, "channels": channels, "rules": rules,
            "params": [float(x) for x in params]}


def product_circuit(n, layers, rng, p1):
    """Layers of U3 (angles U[0, 2pi)) on every qubit, each followed by 1-qubit
    depolarizing p1; no entangling gates, so every trajectory is a product
    state (large-n cases with amplitudes computable one by one)."""
    ops = []
    for layer in range(layers):
        angles = rng.uniform(0.0, 2.0 * math.pi, size=(n, 3))
        for q in range(n):
            ops.append({"kind": "gate", "name": "U3", "qubits": (q,),
                        "params": tuple(float(a) for a in angles[q]), "tag": "U3"})
    channels = [{"name": "depolarizing", "nq": 1, "p": float(p1)}] if p1 > 0 else []
    rules = [{"when": "after_tag", "tag": "U3", "channel": 0}] if p1 > 0 else []
    return {"n_qubits": n, "ops": ops, "channels": channels, "rules": rules, "params": []}


def zz_ring(n):
    """Observable sum_i Z_i Z_{(i+1) mod n} as (coefficient, qubits) Z-strings."""
    return [(1.0, (i, (i + 1) % n)) for i in range(n)]


def _rng(seed, cfg):
    return np.random.default_rng([seed, cfg])


def c1_workload(seed=0):
    """10 qubits, 20 brick layers, p1=1e-3, p2=1e-2; 64 proportional draws x 1000 shots, complex128."""
    circ = brick_circuit(10, 20, _rng(seed, 1), 1e-3, 1e-2)
    return {"name": "C1 10q x 20 brick layers, 64 draws x 1000 shots, complex128", "cfg": 1,
            "seed": seed, "circuit": circ, "precision": "c128",
            "pts": {"mode": "proportional", "n_draws": 64, "total_shots": 64 * 1000,
                    "alloc": "multiplicity"}}


def c2_workload(seed=0, n_draws=512, total_shots=10**6):
    """20 qubits, 40 brick layers, p1=1e-3, p2=5e-3, coherent RZ(eps) per CZ with
    eps ~ N(0, 0.01^2); 512 proportional draws sharing 10^6 shots, complex64."""
    circ = brick_circuit(20, 40, _rng(seed, 2), 1e-3, 5e-3, eps_sigma=0.01)
    return {"name": "C2 20q x 40 brick layers, 512 draws, 1e6 shots, complex64", "cfg": 2,
            "seed": seed, "circuit": circ, "precision": "c64",
            "pts": {"mode": "proportional", "n_draws": n_draws, "total_shots": total_shots,
                    "alloc": "multiplicity"}}


def c3_workload(seed=0, k_max=4096, total_shots=10**9, rounds=5):
    """Rotated d=3 surface-code memory (17 qubits), 5 rounds, p=1e-3; most-likely-first
    enumeration of 4096 Kraus combinations sharing 10^9 shots, complex64."""
    circ = surface_code_d3(rounds=rounds)
    return {"name": "C3 surface code d=3, 5 rounds, top-4096 records, 1e9 shots, complex64",
            "cfg": 3, "seed": seed, "circuit": circ, "precision": "c64",
            "pts": {"mode": "most_likely", "k_max": k_max, "total_shots": total_shots,
                    "alloc": "reweight"}}


def c4_workload(n, seed=0, shots_per_draw=10**5):
    """Brick circuit at n in {24, 26, 28} (30 layers, p2=1e-2, p1=0) with
    256/64/16 draws x 1e5 shots; n = 33 and 35 are one draw x 1e6 shots."""
    draws = {24: 256, 26: 64, 28: 16, 33: 1, 35: 1}.get(n, 16)
    if n in (33, 35):
        shots_per_draw = 10**6
    circ = brick_circuit(n, 30, _rng(seed, 4), 0.0, 1e-2)
    return {"name": f"C4 {n}q x 30 brick layers, {draws} draws x {shots_per_draw} shots, complex64",
            "cfg": 4, "seed": seed, "circuit": circ, "precision": "c64",
            "pts": {"mode": "proportional", "n_draws": draws, "total_shots": draws * shots_per_draw,
                    "alloc": "multiplicity"}}


def c5_workload(seed=0, n=16, layers=8, n_draws=1024):
    """16-qubit hardware-efficient ansatz, 8 layers (256 parameters), p2=5e-3 after
    each ring CZ; 1024 proportional draws; gradient of sum_i Z_i Z_{i+1}."""
    circ = hea_circuit(n, layers, _rng(seed, 5), 5e-3)
    return {"name": f"C5 {n}q HEA x {layers} layers, {n_draws} draws, adjoint gradient",
            "cfg": 5, "seed": seed, "circuit": circ, "precision": "c64",
            "observable": zz_ring(n),
            "pts": {"mode": "proportional", "n_draws": n_draws, "total_shots": n_draws,
                    "alloc": "multiplicity"}}


_ONE_Q = ("H", "X", "Y", "Z", "S", "T")
_ROT = ("RX", "RY", "RZ")


def random_small_circuit(n, n_gates, rng, p1=0.05, p2=0.08, with_params=False,
                         channel_mix=True):
    """A small random circuit for parity tests: random 1- and 2-qubit gates, a
    noise op after many of them (depolarizing, X-flip, asymmetric Pauli, or a
    U3 unitary mixture), optionally parametrised rotations."""
    channels = [
        {"name": "depolarizing", "nq": 1, "p": float(p1)},
        {"name": "depolarizing", "nq": 2, "p": float(p2)},
        {"name": "xflip", "nq": 1, "p": float(p1)},
        {"name": "pauli", "nq": 1, "probs": (0.03, 0.02, 0.05)},
        {"name": "u3_mixture", "nq": 1, "p": 0.07,
         "params": tuple(float(a) for a in rng.uniform(0, 2 * math.pi, 3))},
    ]
    ops = []
    params = []
    for _ in range(n_gates):
        r = rng.random()
        if n >= 2 and r < 0.35:
            a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
            name = ("CZ", "CNOT", "SWAP")[int(rng.integers(3))]
            ops.append({"kind": "gate", "name": name, "qubits": (a, b), "params": (), "tag": name})
            if rng.random() < 0.7:
                ops.append({"kind": "noise", "channel": 1, "qubits": (a, b)})
        else:
            q = int(rng.integers(n))
            if with_params and rng.random() < 0.3:
                gen = ("X", "Y", "Z")[int(rng.integers(3))]
                ops.append({"kind": "param", "gen": gen, "qubits": (q,), "index": len(params),
                            "tag": "R" + gen})
                params.append(float(rng.uniform(0, 2 * math.pi)))
            elif rng.random() < 0.5:
                ops.append({"kind": "gate", "name": "U3", "qubits": (q,),
                            "params": tuple(float(a) for a in rng.uniform(0, 2 * math.pi, 3)),
                            "tag": "U3"})
            elif rng.random() < 0.5:
                name = _ROT[int(rng.integers(3))]
                ops.append({"kind": "gate", "name": name, "qubits": (q,),
                            "params": (float(rng.uniform(0, 2 * math.pi)),), "tag": name})
            else:
                name = _ONE_Q[int(rng.integers(len(_ONE_Q)))]
                ops.append({"kind": "gate", "name": name, "qubits": (q,), "params": (), "tag": name})
            if rng.random() < 0.6:
                ch = int(rng.choice([0, 2, 3, 4])) if channel_mix else 0
                ops.append({"kind": "noise", "channel": ch, "qubits": (q,)})
    return {"n_qubits": n, "ops": ops, "channels": channels, "rules": [], "params": params}
