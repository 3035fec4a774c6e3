"""Fixed-Kraus trajectory preparation in complex128 (Sec. 3, batched execution).

For a trajectory alpha with record {(s, k_s)}, the state is obtained by
applying the circuit's operations in order to |0...0>, with the chosen
operator of every noise site s inserted at its position (k_s = 0 where the
record is silent).  For a unitary-mixture channel the operator applied is the
unitary U_k = K_k / sqrt(p_k); its probability p_k is carried by p_alpha, not
by the state, so the state stays normalised.

Mid-circuit measure-reset is the general (state-dependent) branch of
Algorithm 1 with Kraus pair {|0><0|, |0><1|}: p_1 = sum over x with x_q = 1 of
|psi_x|^2 / ||psi||^2.  Reading used: in the circuits this is applied to
(Clifford circuits with Pauli noise after a projection round) the outcome is
deterministic given the record, so b = [p_1 > 1/2], and
min(p_1, 1 - p_1) must not exceed 1e-6; the state is then projected on b,
renormalised (the K_k / sqrt(p_k) step of Algorithm 1) and reset to |0>.
PROJECT0 applies |0><0| and renormalises.
"""

import math

import numpy as np

from .channels import kraus_ops
from .gates import gate_matrix, rot
from .noise import expand, site_channels
from .rng import key1, uniforms

STREAM_CHANNEL = 4   # uniforms of the state-dependent channel decisions


class NonDeterministicMeasure(RuntimeError):
    pass


def apply(psi, n, mat, qubits):
    """psi <- (mat on qubits) psi by reshape + tensordot (qubit q is axis n-1-q)."""
    k = len(qubits)
    t = psi.reshape((2,) * n)
    m = mat.reshape((2,) * (2 * k))
    # matrix axes 0..k-1 are output bits k-1..0; axes k..2k-1 input bits k-1..0
    in_axes = list(range(k, 2 * k))
    psi_axes = [n - 1 - q for q in reversed(qubits)]
    res = np.tensordot(m, t, axes=(in_axes, psi_axes))
    res = np.moveaxis(res, list(range(k)), psi_axes)
    return np.ascontiguousarray(res).reshape(-1)


def marginal_one(psi, n, q):
    """sum over x with bit q set of |psi_x|^2 (math.fsum) and the total norm^2."""
    p = (psi.real ** 2 + psi.imag ** 2)
    idx = np.arange(psi.size)
    one = math.fsum(p[(idx >> q) & 1 == 1])
    tot = math.fsum(p)
    return one, tot


def zero_state(n):
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def _categorical_positive(u, probs):
    """Smallest k with u < p_0 + ... + p_k (running sum in order, p_k > 0);
    past the end (rounding), the last k with p_k > 0."""
    c = 0.0
    last = 0
    for k, p in enumerate(probs):
        c += p
        if p > 0.0:
            last = k
            if u < c:
                return k
    return last


def run_record(circuit, record, params=None, steps_sites=None, chans=None,
               kraus_unnormalised=False, mr_tol=1e-6, be_key=None, forced=None, trace=None):
    """Prepare psi_alpha for one record.  Returns (psi, mr_bits).

    State-dependent channel steps ("gch") are decided here (Algorithm 1's
    state-dependent branch): p_k = ||K_k psi||^2 / ||psi||^2 on the step's qubits,
    u = word gidx of the stream [seed, key1(4, cfg, alpha)] for ``be_key`` =
    (seed, cfg, alpha), k by the running sum, then K_k / sqrt(p_k); the chosen k
    joins the returned record entries (in record index order with the
    measure-reset bits).  ``forced`` (a list indexed by gidx) fixes the
    decisions instead; if ``trace`` is a list, each decision appends a dict with
    the state before it ("psi"), the qubits, k, p_k and the Kraus operator.

    With ``kraus_unnormalised`` the site operators are K_k = sqrt(p_k) U_k, so
    that ||psi||^2 ends as p_alpha (used as an invariant check)."""
    n = circuit["n_qubits"]
    if steps_sites is None:
        steps_sites = expand(circuit)
    steps, sites = steps_sites
    if chans is None:
        chans = site_channels(circuit)
    if params is None:
        params = circuit.get("params", [])
    ks = dict(record)
    psi = zero_state(n)
    bits = []
    for st in steps:
        kind = st[0]
        if kind == "gate":
            psi = apply(psi, n, gate_matrix(st[1], st[3]), st[2])
        elif kind == "param":
            psi = apply(psi, n, rot(st[1], params[st[3]]), st[2])
        elif kind == "site":
            sid = st[1]
            probs, us = chans[sites[sid]["channel"]]
            k = ks.get(sid, 0)
            U = us[k]
            if kraus_unnormalised:
                U = math.sqrt(probs[k]) * U
            psi = apply(psi, n, U, st[2])
        elif kind == "mr":
            q = st[1][0]
            one, tot = marginal_one(psi, n, q)
            p1 = one / tot
            if min(p1, 1.0 - p1) > mr_tol:
                raise NonDeterministicMeasure(f"measure-reset on qubit {q}: p1 = {p1}")
            b = 1 if p1 > 0.5 else 0
            proj = np.zeros((2, 2), dtype=np.complex128)
            proj[0, b] = 1.0          # |0><b|: project on b, then reset to |0>
            psi = apply(psi, n, proj, (q,))
            psi = psi / math.sqrt(math.fsum(psi.real ** 2 + psi.imag ** 2))
            bits.append(b)
        elif kind == "p0":
            q = st[1][0]
            proj = np.array([[1, 0], [0, 0]], dtype=np.complex128)
            psi = apply(psi, n, proj, (q,))
            psi = psi / math.sqrt(math.fsum(psi.real ** 2 + psi.imag ** 2))
        elif kind == "gch":
            qs = st[1]
            K = kraus_ops(circuit["channels"][st[3]])
            # p_k = <psi|K_k^dagger K_k|psi> / <psi|psi> = ||K_k psi||^2 / ||psi||^2
            tot = math.fsum(psi.real ** 2 + psi.imag ** 2)
            probs = []
            for Kk in K:
                phi = apply(psi, n, Kk, qs)
                probs.append(math.fsum(phi.real ** 2 + phi.imag ** 2) / tot)
            if forced is not None:
                k = forced[st[4]]
            else:
                seed, cfg, alpha = be_key
                u = uniforms(seed, key1(STREAM_CHANNEL, cfg, alpha), st[4] + 1)[st[4]]
                k = _categorical_positive(u, probs)
            if trace is not None:
                trace.append({"psi": psi.copy(), "q": qs, "k": k, "p": probs[k], "K": K[k]})
            psi = apply(psi, n, K[k] / math.sqrt(probs[k]), qs)
            psi = psi / math.sqrt(math.fsum(psi.real ** 2 + psi.imag ** 2))
            bits.append(k)
        else:
            raise ValueError(kind)
    return psi, bits


def product_factors(circuit, record, params=None):
    """One-qubit factors of psi_alpha when every operation and noise site acts on
    a single qubit: then psi = (x)_q v_q with v_q = (product of the operators on
    q, in circuit order) |0>, so amplitude x is prod_q v_q[x_q].  Returns an
    (n, 2) complex128 array; raises ValueError on any multi-qubit step.  This is
    the plain definition of the state for such circuits, usable at any n."""
    n = circuit["n_qubits"]
    steps, sites = expand(circuit)
    chans = site_channels(circuit)
    if params is None:
        params = circuit.get("params", [])
    ks = dict(record)
    v = np.zeros((n, 2), dtype=np.complex128)
    v[:, 0] = 1.0
    for st in steps:
        kind = st[0]
        if kind == "gate":
            U = gate_matrix(st[1], st[3])
        elif kind == "param":
            U = rot(st[1], params[st[3]])
        elif kind == "site":
            _, us = chans[sites[st[1]]["channel"]]
            U = us[ks.get(st[1], 0)]
        else:
            raise ValueError(f"{kind} is not a one-qubit unitary step")
        qs = st[2]
        if len(qs) != 1:
            raise ValueError("product_factors needs one-qubit operations only")
        v[qs[0]] = U @ v[qs[0]]
    return v


def product_amplitudes(factors, xs):
    """Amplitudes <x|psi> = prod_q factors[q, x_q] for basis indices xs."""
    xs = np.asarray(xs, dtype=np.int64)
    out = np.ones(xs.shape, dtype=np.complex128)
    for q in range(factors.shape[0]):
        out *= factors[q, (xs >> q) & 1]
    return out
