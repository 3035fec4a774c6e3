"""Host-side parity of the C++ planner and PTS samplers (through the C ABI, no GPU)
against the oracle: identical site lists and probabilities, identical records,
counts, shot allocations and joint probabilities, bit for bit."""

import numpy as np
import pytest

import paper_2504_16297_amd as P
from oracle.noise import expand, site_probs
from oracle.pts import (alg2_literal, allocate_multiplicity, allocate_reweight, joint_prob,
                        most_likely, proportional, sample_kraus)
from workloads import (c1_workload, c2_workload, c3_workload, c5_workload, random_small_circuit)


def _sites_equal(plan, circ):
    gp, _ = plan.site_probs()
    op = site_probs(circ)
    assert len(gp) == len(op)
    for a, b in zip(gp, op):
        assert list(a) == list(b)          # bitwise: same arithmetic in the same order


@pytest.mark.parametrize("wl", [c1_workload(), c2_workload(), c5_workload()], ids=["C1", "C2", "C5"])
def test_proportional_matches_oracle_on_workloads(wl):
    circ = wl["circuit"]
    plan = P.ptsbe_plan(circ, precision=wl["precision"])
    _sites_equal(plan, circ)
    pts = wl["pts"]
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=pts["n_draws"],
                              total_shots=pts["total_shots"], seed=wl["seed"], cfg=wl["cfg"])
    g = ts.get()
    ref = sample_kraus(site_probs(circ), pts, wl["seed"], wl["cfg"])
    assert g["records"] == ref["records"]
    assert list(g["count"]) == ref["counts"]
    assert list(g["m"]) == ref["m"]
    assert list(g["p"]) == ref["p"]
    assert g["total_shots"] == pts["total_shots"]


@pytest.mark.parametrize("seed", range(5))
def test_random_circuits_all_samplers(seed):
    rng = np.random.default_rng(seed)
    circ = random_small_circuit(int(rng.integers(2, 7)), 40, rng, p1=0.1, p2=0.15)
    plan = P.ptsbe_plan(circ)
    _sites_equal(plan, circ)
    sp = site_probs(circ)
    # proportional
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=300, total_shots=12345, seed=seed, cfg=7)
    g = ts.get()
    recs, counts = proportional(sp, seed, 7, 300)
    assert g["records"] == recs and list(g["count"]) == counts
    assert list(g["m"]) == allocate_multiplicity(counts, 300, 12345)
    # per-shot (Algorithm 1 draws, stream 3, no merging)
    ts = P.ptsbe_sample_kraus(plan, "per_shot", n_draws=50, seed=seed, cfg=7)
    g = ts.get()
    recs, _ = proportional(sp, seed, 7, 50, stream=3, merge=False)
    assert g["records"] == recs and list(g["m"]) == [1] * 50
    # Algorithm 2 as printed
    ts = P.ptsbe_sample_kraus(plan, "alg2_literal", n_draws=200, nshots=17, seed=seed, cfg=7)
    g = ts.get()
    recs, m = alg2_literal(sp, seed, 7, 200, 17)
    assert g["records"] == recs and list(g["m"]) == m
    # most likely first
    for K in (1, 10, 200):
        ts = P.ptsbe_sample_kraus(plan, "most_likely", k_max=K, total_shots=10**6, seed=seed)
        g = ts.get()
        recs, _ = most_likely(sp, K)
        assert g["records"] == recs
        assert list(g["m"]) == allocate_reweight([joint_prob(r, sp) for r in recs], 10**6)
        assert list(g["p"]) == [joint_prob(r, sp) for r in recs]


def test_most_likely_surface_code_top_4096():
    wl = c3_workload()
    circ = wl["circuit"]
    plan = P.ptsbe_plan(circ)
    assert plan.info["n_sites"] == 209 and plan.info["n_measure"] == 40
    _sites_equal(plan, circ)
    ts = P.ptsbe_sample_kraus(plan, "most_likely", k_max=4096, total_shots=10**9)
    g = ts.get()
    sp = site_probs(circ)
    recs, _ = most_likely(sp, 4096)
    assert g["records"] == recs
    assert list(g["m"]) == allocate_reweight([joint_prob(r, sp) for r in recs], 10**9)
    assert int(g["m"].sum()) == 10**9


@pytest.mark.parametrize("mode", ["proportional", "most_likely", "alg2_literal"])
def test_probability_band_matches_oracle(mode):
    """Band PTS (Sec. 3.1): records, draw counts, m_alpha and p_alpha of the
    library equal the oracle's sampler + band filter + allocation, bit for bit."""
    circ = random_small_circuit(4, 30, np.random.default_rng(3), p1=0.1, p2=0.2)
    plan = P.ptsbe_plan(circ)
    sp = site_probs(circ)
    pts = {"proportional": {"mode": "proportional", "n_draws": 400, "total_shots": 4000, "alloc": "multiplicity"},
           "most_likely": {"mode": "most_likely", "k_max": 300, "total_shots": 4000, "alloc": "reweight"},
           "alg2_literal": {"mode": "alg2_literal", "n_draws": 400, "nshots": 9, "alloc": "uniform"}}[mode]
    full = sample_kraus(sp, pts, 1, 2)
    lo, hi = np.quantile(full["p"], [0.25, 0.75])
    ref = sample_kraus(sp, dict(pts, p_band=(lo, hi)), 1, 2)
    tb = P.ptsbe_sample_kraus(plan, mode, n_draws=pts.get("n_draws", 0), k_max=pts.get("k_max", 0),
                              total_shots=pts.get("total_shots", 0), nshots=pts.get("nshots", 0), seed=1, cfg=2,
                              alloc=pts["alloc"], p_band=(lo, hi))
    gb = tb.get()
    assert gb["records"] == ref["records"]
    assert list(gb["count"]) == list(ref["counts"])
    assert list(gb["m"]) == list(ref["m"])
    assert list(gb["p"]) == list(ref["p"])
    assert all(lo <= p <= hi for p in gb["p"])


def test_trajset_slices_and_caller_records():
    circ = random_small_circuit(4, 30, np.random.default_rng(3), p1=0.1, p2=0.2)
    plan = P.ptsbe_plan(circ)
    sp = site_probs(circ)
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=400, total_shots=4000, seed=1, cfg=2)
    g = ts.get()
    s = ts.slice(5, 9).get()
    assert s["alpha0"] == 5 and s["records"] == g["records"][5:9]
    fr = P.ptsbe_trajset_from_records(plan, g["records"][:3], [7, 8, 9], alpha0=11).get()
    assert fr["records"] == g["records"][:3] and list(fr["m"]) == [7, 8, 9]
    assert list(fr["p"]) == [joint_prob(r, sp) for r in g["records"][:3]]


def test_plan_site_order_matches_expansion():
    circ = c3_workload()["circuit"]
    plan = P.ptsbe_plan(circ)
    _, q = plan.site_probs()
    _, sites = expand(circ)
    for s, row in zip(sites, q):
        assert row[0] == s["qubits"][0]
        if len(s["qubits"]) > 1:
            assert row[1] == s["qubits"][1]
        else:
            assert row[1] == 0xFFFFFFFF


def test_adjoint_register_schedule_terminates():
    """Gradient terms take register bits like 2x2 matrices; a register change
    that brings no new bits must not be repeated (this circuit once made the
    scheduler cycle forever)."""
    import time
    from workloads import random_small_circuit
    circ = random_small_circuit(11, 70, np.random.default_rng(311), p1=0.1, p2=0.15, with_params=True)
    t0 = time.perf_counter()
    plan = P.ptsbe_plan(circ, precision="c64")
    assert time.perf_counter() - t0 < 10
    assert plan.info["n_params"] > 0


@pytest.mark.parametrize("seed", range(3))
def test_selection_criteria_match_oracle(seed):
    """Selection criteria (gate type, location, error type, error count and its
    parity) give the oracle's records, counts, shots and p_alpha in every mode."""
    from oracle.pts import select_records
    rng = np.random.default_rng(50 + seed)
    circ = random_small_circuit(6, 50, rng, p1=0.15, p2=0.2)
    plan = P.ptsbe_plan(circ)
    sp = site_probs(circ)
    flags = P.site_selection(plan, qubits=range(1, 6), ops=range(0, 2 * len(circ["ops"]) // 3), kraus=(1, 2, 5, 7))
    off = np.concatenate([[0], np.cumsum([len(p) for p in sp])])
    allow = {(s, k) for s in range(len(sp)) for k in range(1, len(sp[s])) if flags[off[s] + k]}
    assert 0 < len(allow) < sum(len(p) - 1 for p in sp)
    # the same set from the circuit description: site s is the s-th explicit noise op
    expect, s = set(), 0
    for i, op in enumerate(circ["ops"]):
        if op["kind"] != "noise":
            continue
        if all(1 <= q < 6 for q in op["qubits"]) and i < 2 * len(circ["ops"]) // 3:
            expect |= {(s, k) for k in (1, 2, 5, 7) if k < len(sp[s])}
        s += 1
    assert allow == expect
    for crit in ({}, {"max_errors": 2}, {"min_errors": 1, "parity": "odd"}, {"parity": "even"}):
        kw = dict(kraus_allow=flags, **crit)
        ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=400, total_shots=9999, seed=seed, cfg=3, **kw)
        g = ts.get()
        recs, counts = select_records(*proportional(sp, seed, 3, 400, allow=allow), **crit)
        assert g["records"] == recs and list(g["count"]) == counts
        assert list(g["m"]) == allocate_multiplicity(counts, sum(counts), 9999)
        assert list(g["p"]) == [joint_prob(r, sp) for r in recs]
        ts = P.ptsbe_sample_kraus(plan, "alg2_literal", n_draws=150, nshots=5, seed=seed, cfg=3, **kw)
        recs, _ = alg2_literal(sp, seed, 3, 150, 5, allow=allow)
        recs, _ = select_records(recs, [1] * len(recs), **crit)
        assert ts.get()["records"] == recs
        ts = P.ptsbe_sample_kraus(plan, "most_likely", k_max=40, total_shots=10**5, **kw)
        recs, _ = most_likely(sp, 40, allow=allow, **crit)
        assert ts.get()["records"] == recs


def test_selection_by_gate_type_on_tagged_rules():
    """Errors only after CZ gates (gate type) of the brick circuit whose noise
    comes from tag rules; most-likely and proportional records carry no error
    after a U3."""
    from workloads.circuits import brick_circuit
    circ = brick_circuit(6, 4, np.random.default_rng(2), 0.05, 0.1)
    plan = P.ptsbe_plan(circ)
    sp = site_probs(circ)
    flags = P.site_selection(plan, tags=["CZ"], origins=["after_tag"])
    off = np.concatenate([[0], np.cumsum([len(p) for p in sp])])
    allow = {(s, k) for s in range(len(sp)) for k in range(1, len(sp[s])) if flags[off[s] + k]}
    two_q = {s for s in range(len(sp)) if len(sp[s]) == 16}
    assert {s for s, _ in allow} == two_q           # CZ sites are the 2-qubit depolarizing ones
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=300, total_shots=3000, seed=4, cfg=2, kraus_allow=flags)
    recs, counts = proportional(sp, 4, 2, 300, allow=allow)
    assert ts.get()["records"] == recs and all(s in two_q for r in recs for s, _ in r)
    ts = P.ptsbe_sample_kraus(plan, "most_likely", k_max=25, total_shots=10**4, kraus_allow=flags)
    assert ts.get()["records"] == most_likely(sp, 25, allow=allow)[0]


def test_pauli_twirl_matches_oracle_and_plans_twirled_channels():
    """ptsbe_pauli_twirl against the oracle's definition on random CPTP channels,
    and a plan with PTSBE_PLAN_TWIRL: its sites carry the twirled channel's
    probabilities (the plain plan resolves the channel on the device)."""
    from oracle.channels import pauli_twirl, twirled
    rng = np.random.default_rng(21)
    for nq, nk in ((1, 2), (1, 4), (2, 3)):
        d = 2 ** nq
        a = rng.normal(size=(nk * d, d)) + 1j * rng.normal(size=(nk * d, d))
        q, _ = np.linalg.qr(a)
        K = [q[k * d:(k + 1) * d, :] for k in range(nk)]
        got = P.pauli_twirl({"kraus": K})
        assert np.allclose(got, pauli_twirl(K), rtol=0, atol=1e-14)
    ad = {"name": "amplitude_damping", "gamma": 0.3, "nq": 1}
    circ = {"n_qubits": 3, "channels": [ad], "rules": [{"when": "after_tag", "tag": "H", "channel": 0}],
            "params": [], "ops": [{"kind": "gate", "name": "H", "qubits": (q,), "params": (), "tag": "H"}
                                  for q in range(3)]}
    plain = P.ptsbe_plan(circ)            # resolved on the device instead: no pre-sampled site
    assert plain.info["n_sites"] == 0 and plain.info["n_measure"] == 3
    plan = P.ptsbe_plan(circ, twirl=True)
    ref = site_probs(dict(circ, channels=[twirled(ad)]))
    got, _ = plan.site_probs()
    assert len(got) == 3 and all(np.allclose(a, b, rtol=0, atol=1e-15) for a, b in zip(got, ref))


def test_state_dependent_channels_in_forward_and_reverse_programs():
    """Amplitude damping after every RY of a parametrised ansatz: the forward
    program decides each such channel alone (one record entry per decision
    step), and the reverse-sweep program restores them in the opposite order
    (one restore step per channel), so the plan has an adjoint program."""
    from paper_2504_16297_amd.tables import export_adjoint_tables, export_tables
    from workloads.circuits import hea_circuit
    circ = hea_circuit(6, 2, np.random.default_rng(3), 2e-2)
    circ["channels"].append({"name": "amplitude_damping", "gamma": 0.2, "nq": 1})
    circ["rules"].append({"when": "after_tag", "tag": "RY", "channel": 1})
    params = np.asarray(circ["params"])
    for tile in (0, 5):
        plan = P.ptsbe_plan(circ, tile_qubits=tile)
        info = plan.record_info()
        gch = [r for r, (c, _) in enumerate(info) if c >= 0]
        assert len(gch) == 12 and plan.info["n_measure"] == 12
        ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=8, total_shots=8, seed=1, cfg=1)
        fwd = export_tables(ts, params)
        dec = [list(e["idx"][:e["nq"]]) for e in fwd["exec"] if e["pass"] == 0xFFFFFFFF]
        assert dec == [[r] for r in gch]
        adj, _ = export_adjoint_tables(ts, params)
        res = [list(e["idx"][:e["nq"]]) for e in adj["exec"] if e["pass"] == 0xFFFFFFFF]
        assert res == [[r] for r in reversed(gch)]


def test_autotune_candidates():
    """The tuner's candidates: the two largest register-kernel tiles that fit,
    fill 2 or 3, whole or half-tile register changes, pair fusion on or off;
    each builds a plan."""
    from paper_2504_16297_amd.tune import candidates_for
    c = candidates_for(20, "c64")
    assert len(c) == 16 and len(set(c)) == 16
    assert {t for t, _, _, _ in c} == {12, 11} and {pf for _, _, _, pf in c} == {True, False}
    assert {t for t, _, _, _ in candidates_for(11, "c64")} == {11, 10}
    assert {t for t, _, _, _ in candidates_for(20, "c128")} == {11, 10}
    assert {t for t, _, _, _ in candidates_for(4, "c64")} == {0}
    circ = random_small_circuit(8, 30, np.random.default_rng(2))
    for tile, fill, half, pf in candidates_for(8, "c64"):
        P.ptsbe_plan(circ, tile_qubits=tile, min_fill=fill, half_tile=half, pair_fusion=pf)


def test_tuning_cache_keys_and_reuse(tmp_path, monkeypatch):
    """The autotuner's cache: a miss tunes once and stores the pick under a key
    of the circuit and precision; a hit returns it without
    tuning; another circuit or precision is another key."""
    from paper_2504_16297_amd import tune
    calls = []

    def fake_autotune(circuit, precision="c64", **kw):
        calls.append((circuit["n_qubits"], precision))
        return {"tile_qubits": 11, "min_fill": 3, "half_tile": False, "pair_fusion": True,
                "results": [(11, 3, False, True, 1.5, 0.1)], "seconds": 0.2}

    monkeypatch.setattr(tune, "autotune", fake_autotune)
    cache = str(tmp_path / "tune.json")
    a = random_small_circuit(8, 30, np.random.default_rng(1))
    b = random_small_circuit(8, 30, np.random.default_rng(2))
    assert tune.tuned_plan_options(a, "c64", cache=cache) == (None, None)
    opts, e = tune.tuned_plan_options(a, "c64", cache=cache, tune_if_missing=True)
    assert opts == {"tile_qubits": 11, "min_fill": 3, "half_tile": False, "pair_fusion": True}
    assert tune.tuned_plan_options(a, "c64", cache=cache)[0] == opts and len(calls) == 1
    assert tune.tuned_plan_options(b, "c64", cache=cache)[0] is None
    assert tune.tuned_plan_options(a, "c128", cache=cache)[0] is None
    plan = P.ptsbe_plan(a, **opts)
    assert plan.info["tile_qubits"] == 8      # tiles are capped at the qubit count
