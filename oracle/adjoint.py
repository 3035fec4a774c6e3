"""Expectation values and adjoint gradients of the trajectory ensemble.

Pre-trajectory sampling fixes every trajectory's Kraus choices before
execution (Sec. 3), so each trajectory is a deterministic circuit and the
ensemble estimate of <O> is E(theta) = sum_alpha w_alpha <psi_alpha|O|psi_alpha>
with w_alpha = count_alpha / T.  For unitary-mixture channels w_alpha does not
depend on theta, so grad E = sum_alpha w_alpha grad <O>_alpha.

Adjoint method (reverse sweep): lambda = O psi; for each operation G in reverse,
psi <- G^dagger psi; if G = exp(-i theta P / 2) add
2 Re <lambda| dG/dtheta |psi>; lambda <- G^dagger lambda.
O is a sum of Z-strings, hence diagonal.

State-dependent channels (Algorithm 1's state-dependent branch): a trajectory
also carries the Kraus choices k drawn with p_k = ||K_k psi||^2 when its state
reached each such channel.  For the unnormalised path state phi (raw K_k), the
ensemble value is sum over paths of <phi|O|phi>, so its derivative is the
average over drawn paths of d<phi|O|phi> / <phi|phi>.  That equals the adjoint
sweep of the normalised trajectory with every chosen G = K_k / sqrt(p_k) held
fixed (the pathwise derivative of <O>_psi plus <O>_psi d log p(path), the
score-function term, together).  A singular K_k cannot be un-applied, so the
sweep takes psi back from the state recorded before the channel and applies
G^dagger to lambda alone.
"""

import numpy as np

from .gates import gate_matrix, rot, rot_derivative
from .noise import expand, site_channels
from .statevector import apply, run_record


def observable_diag(n, terms):
    """Diagonal of sum_t coef_t prod_{q in t} Z_q."""
    x = np.arange(1 << n)
    d = np.zeros(1 << n, dtype=np.float64)
    for coef, qs in terms:
        sign = np.ones(1 << n)
        for q in qs:
            sign = sign * (1 - 2 * ((x >> q) & 1))
        d += coef * sign
    return d


def expval(psi, odiag):
    w = psi.real ** 2 + psi.imag ** 2
    return float(np.sum(w * odiag))


def trajectory_grad(circuit, record, params, odiag, steps_sites=None, chans=None, be_key=None, forced=None):
    """(<O>_alpha, d<O>_alpha/dparams) for one record by the adjoint sweep;
    state-dependent channels decided by ``be_key`` or ``forced`` as in
    run_record, with their chosen operators held fixed."""
    n = circuit["n_qubits"]
    if steps_sites is None:
        steps_sites = expand(circuit)
    steps, sites = steps_sites
    if chans is None:
        chans = site_channels(circuit)
    trace = []
    psi, _ = run_record(circuit, record, params=params, steps_sites=steps_sites, chans=chans,
                        be_key=be_key, forced=forced, trace=trace)
    e = expval(psi, odiag)
    lam = odiag * psi
    grad = np.zeros(len(params))
    ks = dict(record)
    for st in reversed(steps):
        kind = st[0]
        if kind == "gate":
            U = gate_matrix(st[1], st[3])
            Ud = U.conj().T
            psi = apply(psi, n, Ud, st[2])
            lam = apply(lam, n, Ud, st[2])
        elif kind == "site":
            _, us = chans[sites[st[1]]["channel"]]
            Ud = us[ks.get(st[1], 0)].conj().T
            psi = apply(psi, n, Ud, st[2])
            lam = apply(lam, n, Ud, st[2])
        elif kind == "param":
            theta = params[st[3]]
            Gd = rot(st[1], theta).conj().T
            psi = apply(psi, n, Gd, st[2])
            mu = apply(psi, n, rot_derivative(st[1], theta), st[2])
            grad[st[3]] += 2.0 * np.real(np.vdot(lam, mu))
            lam = apply(lam, n, Gd, st[2])
        elif kind == "gch":
            d = trace[st[4]]
            G = d["K"] / np.sqrt(d["p"])
            psi = d["psi"]
            lam = apply(lam, n, G.conj().T, d["q"])
        else:
            raise ValueError(f"adjoint does not support {kind}")
    return e, grad


def ensemble_value_and_grad(circuit, records, weights, params, terms, be_seed=None):
    """Weighted ensemble value and gradient; with ``be_seed`` = (seed, cfg),
    trajectory a's state-dependent channels are decided with key (seed, cfg, a)."""
    n = circuit["n_qubits"]
    odiag = observable_diag(n, terms)
    ss = expand(circuit)
    chans = site_channels(circuit)
    E = 0.0
    G = np.zeros(len(params))
    for a, (rec, w) in enumerate(zip(records, weights)):
        key = None if be_seed is None else (be_seed[0], be_seed[1], a)
        e, g = trajectory_grad(circuit, rec, params, odiag, ss, chans, be_key=key)
        E += w * e
        G += w * g
    return E, G


def ensemble_value(circuit, records, weights, params, terms):
    n = circuit["n_qubits"]
    odiag = observable_diag(n, terms)
    ss = expand(circuit)
    chans = site_channels(circuit)
    E = 0.0
    for rec, w in zip(records, weights):
        psi, _ = run_record(circuit, rec, params=params, steps_sites=ss, chans=chans)
        E += w * expval(psi, odiag)
    return E


def parameter_shift(circuit, records, weights, params, terms):
    """dE/dtheta_i = [E(theta_i + pi/2) - E(theta_i - pi/2)] / 2, exact for exp(-i theta P/2)."""
    params = np.asarray(params, dtype=np.float64)
    g = np.zeros(params.size)
    for i in range(params.size):
        pp = params.copy(); pp[i] += np.pi / 2
        pm = params.copy(); pm[i] -= np.pi / 2
        g[i] = 0.5 * (ensemble_value(circuit, records, weights, pp, terms)
                      - ensemble_value(circuit, records, weights, pm, terms))
    return g
