"""Pins of the oracle's state-dependent channels (amplitude damping resolved
when the state reaches it, Algorithm 1's state-dependent branch): hand-worked
decisions on |0> and |1>, and the average over many trajectories of
|psi><psi| against the exact density matrix."""

import math

import numpy as np

from oracle.densitymatrix import evolve
from oracle.noise import expand
from oracle.rng import key1, uniforms
from oracle.statevector import run_record


def _circ(ops, gamma=0.3, n=1):
    return {"n_qubits": n, "ops": ops, "params": [], "rules": [],
            "channels": [{"name": "amplitude_damping", "gamma": gamma, "nq": 1}]}


def test_steps_and_record_indices():
    c = _circ([{"kind": "gate", "name": "X", "qubits": (0,), "params": (), "tag": "X"},
               {"kind": "noise", "channel": 0, "qubits": (0,)},
               {"kind": "measure_reset", "qubits": (0,)},
               {"kind": "noise", "channel": 0, "qubits": (0,)}])
    steps, sites = expand(c)
    assert sites == []
    assert [s[0] for s in steps] == ["gate", "gch", "mr", "gch"]
    assert [s[2] for s in steps if s[0] in ("gch", "mr")] == [0, 1, 2]   # one record index counter
    assert [s[4] for s in steps if s[0] == "gch"] == [0, 1]


def test_hand_worked_decisions():
    g = 0.3
    one = _circ([{"kind": "gate", "name": "X", "qubits": (0,), "params": (), "tag": "X"},
                 {"kind": "noise", "channel": 0, "qubits": (0,)}], gamma=g)
    zero = _circ([{"kind": "noise", "channel": 0, "qubits": (0,)}], gamma=g)
    for alpha in range(40):
        u = uniforms(5, key1(4, 2, alpha), 1)[0]
        psi, rec = run_record(one, (), be_key=(5, 2, alpha))
        # from |1>: p = (1 - g, g); k = 0 keeps |1>, k = 1 decays to |0>
        assert rec == [0 if u < 1 - g else 1]
        assert np.allclose(np.abs(psi), [0, 1] if rec[0] == 0 else [1, 0])
        psi, rec = run_record(zero, (), be_key=(5, 2, alpha))
        assert rec == [0] and np.allclose(psi, [1, 0])              # |0> never decays


def test_trajectory_average_equals_density_matrix():
    c = {"n_qubits": 3, "params": [],
         "channels": [{"name": "amplitude_damping", "gamma": 0.35, "nq": 1},
                      {"name": "depolarizing", "nq": 1, "p": 0.0}],
         "rules": [{"when": "after_tag", "tag": "H", "channel": 0}, {"when": "after_tag", "tag": "RX", "channel": 0}],
         "ops": [{"kind": "gate", "name": "H", "qubits": (0,), "params": (), "tag": "H"},
                 {"kind": "gate", "name": "CNOT", "qubits": (0, 1), "params": (), "tag": "CX"},
                 {"kind": "gate", "name": "RX", "qubits": (2,), "params": (1.1,), "tag": "RX"},
                 {"kind": "gate", "name": "H", "qubits": (2,), "params": (), "tag": "H"},
                 {"kind": "gate", "name": "CNOT", "qubits": (2, 1), "params": (), "tag": "CX"}]}
    rho = evolve(c)
    T = 4000
    acc = np.zeros_like(rho)
    for alpha in range(T):
        psi, _ = run_record(c, (), be_key=(11, 7, alpha))
        acc += np.outer(psi, psi.conj())
    acc /= T
    err = float(np.max(np.abs(acc - rho)))
    assert err < 5 * 0.5 / math.sqrt(T), err


def test_channel_diagonals_closed_form():
    from oracle.channels import general_channel, kraus_ops
    g = 0.3
    # amplitude damping: K0 = diag(1, sqrt(1-g)), K1 = sqrt(g)|0><1|
    # K0^dag K0 = diag(1, 1-g), K1^dag K1 = diag(0, g)
    d0, d1 = general_channel(kraus_ops({"name": "amplitude_damping", "gamma": g, "nq": 1}))
    assert np.allclose(d0, [1.0, 0.0]) and np.allclose(d1, [1.0 - g, g])
    # a channel whose K^dag K is not diagonal has no such form
    h = np.array([[1, 1], [1, -1]]) / math.sqrt(2)
    off = [math.sqrt(0.5) * np.eye(2), math.sqrt(0.5) * h @ np.diag([1.0, 0.0]) @ h,
           math.sqrt(0.5) * h @ np.diag([0.0, 1.0]) @ h]
    assert general_channel(off) is None


def _ad_hea(gamma=0.25):
    """3-qubit, 2-layer RY/RZ ansatz with CZ ring; amplitude damping after every RY."""
    ops = []
    for layer in range(2):
        for q in range(3):
            b = layer * 6 + 2 * q
            ops.append({"kind": "param", "gen": "Y", "qubits": (q,), "index": b, "tag": "RY"})
            ops.append({"kind": "param", "gen": "Z", "qubits": (q,), "index": b + 1, "tag": "RZ"})
        for i in range(3):
            ops.append({"kind": "gate", "name": "CZ", "qubits": (i, (i + 1) % 3), "params": (), "tag": "CZ"})
    params = np.random.default_rng(21).uniform(0.0, 2.0 * math.pi, size=12)
    return {"n_qubits": 3, "ops": ops, "params": [float(x) for x in params],
            "channels": [{"name": "amplitude_damping", "gamma": gamma, "nq": 1}],
            "rules": [{"when": "after_tag", "tag": "RY", "channel": 0}]}


def _paths(circ, params, terms):
    """Every decision path with its probability (product of the p_k met),
    value and fixed-operator adjoint gradient."""
    import itertools
    from oracle.adjoint import observable_diag, trajectory_grad
    n_gch = sum(1 for s in expand(circ)[0] if s[0] == "gch")
    od = observable_diag(circ["n_qubits"], terms)
    out = []
    for path in itertools.product(range(2), repeat=n_gch):
        tr = []
        run_record(circ, (), params=params, forced=list(path), trace=tr)
        prob = math.prod(d["p"] for d in tr)
        e, g = trajectory_grad(circ, (), params, od, forced=list(path))
        out.append((path, prob, e, g))
    return out


def test_gradient_through_channels_sums_to_density_matrix_derivative():
    """sum over all decision paths of p(path) * (fixed-operator adjoint gradient)
    equals the derivative of Tr(O rho(theta)) under the full channel (parameter
    shift of the density-matrix evolution); a gradient without the score-function
    part (each path's derivative of its normalised expectation) does not."""
    circ = _ad_hea()
    p = np.asarray(circ["params"])
    terms = [(1.0, (0, 1)), (0.6, (2,)), (-0.4, (0,))]
    from oracle.adjoint import observable_diag
    od = observable_diag(3, terms)

    def exact(pp):
        return float(np.real(np.sum(np.diag(evolve(circ, pp)) * od)))

    paths = _paths(circ, p, terms)
    assert abs(sum(pr for _, pr, _, _ in paths) - 1.0) < 1e-12
    assert abs(sum(pr * e for _, pr, e, _ in paths) - exact(p)) < 1e-12
    G = sum(pr * g for _, pr, _, g in paths)
    shift = np.zeros(p.size)
    for i in range(p.size):
        pp = p.copy(); pp[i] += math.pi / 2
        pm = p.copy(); pm[i] -= math.pi / 2
        shift[i] = 0.5 * (exact(pp) - exact(pm))
    assert float(np.max(np.abs(G - shift))) < 1e-11
    # the pathwise part alone (derivative of <O> along each fixed path) misses the
    # score-function term, and the sum then differs from the exact derivative
    h = 1e-5
    pathwise = np.zeros(p.size)
    for path, pr, _, _ in paths:
        for i in range(p.size):
            pp = p.copy(); pp[i] += h
            pm = p.copy(); pm[i] -= h
            ep = float(np.sum(np.abs(run_record(circ, (), params=pp, forced=list(path))[0]) ** 2 * od))
            em = float(np.sum(np.abs(run_record(circ, (), params=pm, forced=list(path))[0]) ** 2 * od))
            pathwise[i] += pr * (ep - em) / (2 * h)
    assert float(np.max(np.abs(pathwise - shift))) > 1e-3


def test_path_gradient_is_derivative_of_unnormalised_value():
    """For one fixed path, the adjoint gradient equals d<phi|O|phi>/dtheta divided
    by <phi|phi> (phi: the path state under the raw Kraus operators; <phi|phi>
    = p(path), <phi|O|phi> = p(path) <O>), by central differences."""
    circ = _ad_hea(0.4)
    p = np.asarray(circ["params"])
    terms = [(1.0, (1, 2)), (0.3, (0,))]
    from oracle.adjoint import observable_diag, trajectory_grad
    od = observable_diag(3, terms)
    path = [1, 0, 1, 0, 0, 1]

    def f(pp):
        tr = []
        psi, _ = run_record(circ, (), params=pp, forced=path, trace=tr)
        return math.prod(d["p"] for d in tr) * float(np.sum(np.abs(psi) ** 2 * od)), math.prod(d["p"] for d in tr)

    _, g = trajectory_grad(circ, (), p, od, forced=path)
    _, prob = f(p)
    h = 1e-5
    for i in range(p.size):
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        fd = (f(pp)[0] - f(pm)[0]) / (2 * h) / prob
        assert abs(fd - g[i]) < 1e-7, (i, fd, g[i])


# --- channels whose K^dagger K are not diagonal, and two-qubit channels

def _rotated_damping(g, theta):
    """Amplitude damping conjugated by RY(theta): K_k^dagger K_k not diagonal."""
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    U = np.array([[c, -s], [s, c]], dtype=np.complex128)
    K0 = np.array([[1, 0], [0, math.sqrt(1 - g)]], dtype=np.complex128)
    K1 = np.array([[0, math.sqrt(g)], [0, 0]], dtype=np.complex128)
    return [U @ K0 @ U.conj().T, U @ K1 @ U.conj().T]


def _pair_decay(g):
    """Two-qubit joint decay |11> -> |00> with probability g (not a unitary mixture):
    K0 = diag(1, 1, 1, sqrt(1-g)), K1 = sqrt(g) |00><11|."""
    K0 = np.diag([1.0, 1.0, 1.0, math.sqrt(1 - g)]).astype(np.complex128)
    K1 = np.zeros((4, 4), dtype=np.complex128)
    K1[0, 3] = math.sqrt(g)
    return [K0, K1]


def test_state_dependent_channel_classes():
    from oracle.channels import cptp_error, general_channel, state_dependent
    rd = _rotated_damping(0.3, 0.8)
    pd = _pair_decay(0.4)
    for K in (rd, pd):
        assert cptp_error(K) < 1e-14 and state_dependent(K)
    assert general_channel(rd) is None and general_channel(pd) is None
    # unitary mixtures are pre-sampled, not state dependent
    from oracle.channels import kraus_ops
    assert not state_dependent(kraus_ops({"name": "depolarizing", "nq": 2, "p": 0.1}))


def test_pair_decay_hand_worked():
    """From |11> the joint decay happens with probability g (u >= 1 - g) and
    leaves |00>; from |01> it never happens."""
    g = 0.35
    c = {"n_qubits": 2, "params": [], "rules": [], "channels": [{"kraus": _pair_decay(g), "nq": 2}],
         "ops": [{"kind": "gate", "name": "X", "qubits": (0,), "params": (), "tag": "X"},
                 {"kind": "gate", "name": "X", "qubits": (1,), "params": (), "tag": "X"},
                 {"kind": "noise", "channel": 0, "qubits": (0, 1)}]}
    c01 = dict(c, ops=c["ops"][:1] + c["ops"][2:])
    for alpha in range(40):
        u = uniforms(3, key1(4, 1, alpha), 1)[0]
        psi, rec = run_record(c, (), be_key=(3, 1, alpha))
        assert rec == [0 if u < 1 - g else 1]
        assert np.allclose(np.abs(psi), [0, 0, 0, 1] if rec[0] == 0 else [1, 0, 0, 0])
        psi, rec = run_record(c01, (), be_key=(3, 1, alpha))
        assert rec == [0] and np.allclose(np.abs(psi), [0, 1, 0, 0])


def _dense_circuit():
    return {"n_qubits": 3, "params": [],
            "channels": [{"kraus": _rotated_damping(0.45, 0.9), "nq": 1}, {"kraus": _pair_decay(0.5), "nq": 2}],
            "rules": [{"when": "after_tag", "tag": "H", "channel": 0}, {"when": "after_tag", "tag": "CX", "channel": 1}],
            "ops": [{"kind": "gate", "name": "H", "qubits": (0,), "params": (), "tag": "H"},
                    {"kind": "gate", "name": "CNOT", "qubits": (0, 1), "params": (), "tag": "CX"},
                    {"kind": "gate", "name": "RX", "qubits": (2,), "params": (1.1,), "tag": "RX"},
                    {"kind": "gate", "name": "H", "qubits": (2,), "params": (), "tag": "H"},
                    {"kind": "gate", "name": "CNOT", "qubits": (2, 1), "params": (), "tag": "CX"}]}


def test_dense_channels_trajectory_average_equals_density_matrix():
    """1-qubit channels with non-diagonal K^dagger K and a 2-qubit channel, each
    decided from the state: the average of |psi><psi| over trajectories is the
    density-matrix evolution under the full channels, and the exact average over
    every decision path with its probability equals it to rounding."""
    import itertools
    c = _dense_circuit()
    rho = evolve(c)
    n_gch = sum(1 for s in expand(c)[0] if s[0] == "gch")
    exact = np.zeros_like(rho)
    for path in itertools.product(range(2), repeat=n_gch):
        tr = []
        with np.errstate(divide="ignore", invalid="ignore"):
            psi, _ = run_record(c, (), forced=list(path), trace=tr)
        pr = math.prod(d["p"] for d in tr)
        if pr > 0.0:
            exact += pr * np.outer(psi, psi.conj())
    assert float(np.max(np.abs(exact - rho))) < 1e-12
    T = 3000
    acc = np.zeros_like(rho)
    for alpha in range(T):
        psi, _ = run_record(c, (), be_key=(17, 2, alpha))
        acc += np.outer(psi, psi.conj())
    acc /= T
    assert float(np.max(np.abs(acc - rho))) < 5 * 0.5 / math.sqrt(T)


def test_dense_channel_gradient_sums_to_density_matrix_derivative():
    """Over all decision paths, sum of p(path) times the fixed-operator adjoint
    gradient equals the parameter shift of Tr(O rho(theta)) with the 1-qubit
    non-diagonal and the 2-qubit channels."""
    import itertools
    from oracle.adjoint import observable_diag, trajectory_grad
    ops = []
    for layer in range(2):
        for q in range(3):
            ops.append({"kind": "param", "gen": "Y", "qubits": (q,), "index": 2 * (3 * layer + q), "tag": "RY"})
            ops.append({"kind": "param", "gen": "Z", "qubits": (q,), "index": 2 * (3 * layer + q) + 1, "tag": "RZ"})
        ops.append({"kind": "gate", "name": "CZ", "qubits": (0, 1), "params": (), "tag": "CZ"})
        ops.append({"kind": "gate", "name": "CZ", "qubits": (1, 2), "params": (), "tag": "CZ"})
    params = np.random.default_rng(8).uniform(0, 2 * math.pi, 12)
    c = {"n_qubits": 3, "ops": ops, "params": [float(x) for x in params],
         "channels": [{"kraus": _rotated_damping(0.3, 0.7), "nq": 1}, {"kraus": _pair_decay(0.4), "nq": 2}],
         "rules": [{"when": "after_tag", "tag": "RY", "channel": 0}, {"when": "after_tag", "tag": "CZ", "channel": 1}]}
    terms = [(1.0, (0, 1)), (0.5, (2,)), (-0.3, (1,))]
    od = observable_diag(3, terms)
    n_gch = sum(1 for s in expand(c)[0] if s[0] == "gch")

    def exact(pp):
        return float(np.real(np.sum(np.diag(evolve(c, pp)) * od)))

    G = np.zeros(params.size)
    total = 0.0
    for path in itertools.product(range(2), repeat=n_gch):
        tr = []
        with np.errstate(divide="ignore", invalid="ignore"):
            run_record(c, (), params=params, forced=list(path), trace=tr)
        pr = math.prod(d["p"] for d in tr)
        if not pr > 0.0:     # a path through a zero-probability operator (e.g. a decay of |00>)
            continue
        total += pr
        _, g = trajectory_grad(c, (), params, od, forced=list(path))
        G += pr * g
    assert abs(total - 1.0) < 1e-12
    shift = np.zeros(params.size)
    for i in range(params.size):
        pp = params.copy(); pp[i] += math.pi / 2
        pm = params.copy(); pm[i] -= math.pi / 2
        shift[i] = 0.5 * (exact(pp) - exact(pm))
    assert float(np.max(np.abs(G - shift))) < 1e-11
