"""Pins of the oracle's density-matrix evolution on its measure-reset and
PROJECT0 branches (the general, state-dependent branch of Algorithm 1 and the
projection that prepares a code state): hand-worked small cases, and the
exhaustive trajectory ensemble of circuits whose mid-circuit outcomes are
deterministic given the record."""

import itertools
import math

import numpy as np

from oracle.densitymatrix import evolve
from oracle.noise import expand, site_channels, site_probs
from oracle.pts import joint_prob
from oracle.statevector import run_record


def _g(name, qubits, params=()):
    return {"kind": "gate", "name": name, "qubits": tuple(qubits), "params": tuple(params), "tag": name}


def _circ(n, ops, channels=(), rules=()):
    return {"n_qubits": n, "ops": list(ops), "channels": list(channels), "rules": list(rules), "params": []}


def test_measure_reset_of_one_qubit():
    # |+> measured and reset: both outcomes end in |0>
    rho = evolve(_circ(1, [_g("H", (0,)), {"kind": "measure_reset", "qubits": (0,)}]))
    assert np.allclose(rho, [[1, 0], [0, 0]], atol=1e-15)
    # |1> measured and reset: |0>
    rho = evolve(_circ(1, [_g("X", (0,)), {"kind": "measure_reset", "qubits": (0,)}]))
    assert np.allclose(rho, [[1, 0], [0, 0]], atol=1e-15)


def test_measure_reset_of_half_a_bell_pair():
    # (|00> + |11>)/sqrt 2 (index x = x0 + 2 x1), measure-reset qubit 1:
    # outcome 0 keeps |00>, outcome 1 sends |11> to |x0=1, x1=0> = index 1; the
    # coherence between them is gone: rho = diag(1/2, 1/2, 0, 0)
    circ = _circ(2, [_g("H", (0,)), _g("CNOT", (0, 1)), {"kind": "measure_reset", "qubits": (1,)}])
    rho = evolve(circ)
    assert np.allclose(rho, np.diag([0.5, 0.5, 0.0, 0.0]), atol=1e-15)
    # measure-reset of qubit 0 instead: |00> stays, |11> -> |x0=0, x1=1> = index 2
    circ = _circ(2, [_g("H", (0,)), _g("CNOT", (0, 1)), {"kind": "measure_reset", "qubits": (0,)}])
    assert np.allclose(evolve(circ), np.diag([0.5, 0.0, 0.5, 0.0]), atol=1e-15)


def test_measure_reset_keeps_the_other_qubits_coherence():
    # |+>|1> (q0 = +, q1 = 1): resetting q1 leaves |+>|0>, a pure state
    circ = _circ(2, [_g("H", (0,)), _g("X", (1,)), {"kind": "measure_reset", "qubits": (1,)}])
    want = np.zeros((4, 4))
    want[np.ix_([0, 1], [0, 1])] = 0.5
    assert np.allclose(evolve(circ), want, atol=1e-15)


def test_project0_by_hand():
    # |++>, project qubit 1 on |0>: (|00> + |01>)/sqrt 2 in index order x0 + 2 x1 -> indices 0, 1
    circ = _circ(2, [_g("H", (0,)), _g("H", (1,)), {"kind": "project0", "qubits": (1,)}])
    want = np.zeros((4, 4))
    want[np.ix_([0, 1], [0, 1])] = 0.5
    assert np.allclose(evolve(circ), want, atol=1e-15)
    # RY(theta)|0> then |0><0|: the trace cos^2(theta/2) is divided out
    circ = _circ(1, [_g("RY", (0,), (1.1,)), {"kind": "project0", "qubits": (0,)}])
    assert np.allclose(evolve(circ), [[1, 0], [0, 0]], atol=1e-15)
    # entangled: RY(theta) q0, CNOT q0 -> q1, project q0 on |0>: |00>
    circ = _circ(2, [_g("RY", (0,), (2.0,)), _g("CNOT", (0, 1)), {"kind": "project0", "qubits": (0,)}])
    assert np.allclose(evolve(circ), np.diag([1.0, 0, 0, 0]), atol=1e-15)


def test_project0_on_a_mixed_state_renormalises_the_whole_matrix():
    # a depolarized |+> projected on |0>: rho_00 / tr = 1 whatever the noise
    circ = _circ(1, [_g("H", (0,)), {"kind": "noise", "channel": 0, "qubits": (0,)},
                     {"kind": "project0", "qubits": (0,)}],
                 channels=[{"name": "depolarizing", "nq": 1, "p": 0.3}])
    assert np.allclose(evolve(circ), [[1, 0], [0, 0]], atol=1e-15)
    # a 2-qubit mixture: X-flip (p) on q1 of |+>|0>, then project q0 on |0>:
    # rho = (1-p)|00><00| + p|0,1><0,1| (index x0 + 2 x1: 0 and 2)
    p = 0.25
    circ = _circ(2, [_g("H", (0,)), {"kind": "noise", "channel": 0, "qubits": (1,)},
                     {"kind": "project0", "qubits": (0,)}],
                 channels=[{"name": "xflip", "nq": 1, "p": p}])
    assert np.allclose(evolve(circ), np.diag([1 - p, 0, p, 0]), atol=1e-15)


def _parity_check_circuit(p_flip, p_dep):
    """Two data qubits in (|00> + |11>)/sqrt 2 (a noiseless prefix with a
    PROJECT0 of the ancilla), then two rounds of a ZZ parity check measured into
    ancilla 2 with measure-reset, X-flips on the data before each round and a
    1-qubit depolarizing site on data qubit 0 after the check gates: Clifford
    gates with Pauli noise, so every outcome is deterministic given the record
    (256 records in all)."""
    ops = [_g("H", (0,)), _g("CNOT", (0, 1)), _g("H", (2,)), {"kind": "project0", "qubits": (2,)}]
    for _ in range(2):
        ops += [{"kind": "noise", "channel": 0, "qubits": (0,)},
                {"kind": "noise", "channel": 0, "qubits": (1,)},
                _g("CNOT", (0, 2)), _g("CNOT", (1, 2)),
                {"kind": "noise", "channel": 1, "qubits": (0,)},
                {"kind": "measure_reset", "qubits": (2,)}]
    return _circ(3, ops, channels=[{"name": "xflip", "nq": 1, "p": p_flip},
                                   {"name": "depolarizing", "nq": 1, "p": p_dep}])


def test_exhaustive_ensemble_with_measure_resets_equals_density_matrix():
    """sum_alpha p_alpha |psi_alpha><psi_alpha| over every record equals the
    density matrix when each outcome is deterministic given the record: then
    the measure-reset channel maps each trajectory's state to one pure state
    without changing its weight."""
    circ = _parity_check_circuit(0.2, 0.3)
    sp = site_probs(circ)
    ss = expand(circ)
    ch = site_channels(circ)
    rho = evolve(circ)
    acc = np.zeros_like(rho)
    total = 0.0
    seen_one = False
    for ks in itertools.product(*[range(len(p)) for p in sp]):
        rec = tuple((s, k) for s, k in enumerate(ks) if k)
        psi, bits = run_record(circ, rec, steps_sites=ss, chans=ch)
        seen_one |= any(bits)
        pa = joint_prob(rec, sp)
        acc += pa * np.outer(psi, psi.conj())
        total += pa
    assert seen_one                      # some records do flip the recorded parity
    assert math.isclose(total, 1.0, abs_tol=1e-12)
    assert np.max(np.abs(acc - rho)) < 1e-12
    assert abs(np.trace(rho).real - 1.0) < 1e-12


def test_density_matrix_measure_reset_differs_from_dropping_it():
    # the measure-reset branch is not a no-op on the parity circuit
    circ = _parity_check_circuit(0.2, 0.3)
    rho = evolve(circ)
    no_mr = dict(circ, ops=[op for op in circ["ops"] if op["kind"] != "measure_reset"])
    assert np.max(np.abs(evolve(no_mr) - rho)) > 0.1
