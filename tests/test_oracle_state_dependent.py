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
