"""Autotuner of the plan's launch shape.

The tile size k (tile qubits per pass: more qubits per tile means fewer passes
but more LDS per workgroup and so fewer resident workgroups per CU), the
register-group fill threshold (fewer, fuller 2x2 groups against more register
changes), the half-tile register changes (half the LDS, two more barriers
per change) and pair fusion (4x4 slots over the 2x2 runs around a diagonal
2-qubit gate: fewer flops in brick circuits, more where a 4x4 takes in little)
trade against each other differently for every circuit.  `autotune`
builds the plan for each candidate, compiles its passes, runs a sample of the
trajectory set through the library's stage timer on the device, and returns the
candidate with the least tile-pass time on that sample.  Trajectory records are
plan-independent (the noise sites depend only on the circuit), so one sample is
carried across candidates with ptsbe_trajset_from_records.

`tuned_plan_options` keeps the picks in a JSON cache keyed by a hash of the
circuit description and the precision, so a workload is
tuned once per machine (``python -m paper_2504_16297_amd.tune`` fills the
cache for the benchmark workloads); the default cache is the package's
``tune_cache.json``, or the file named by ``PTSBE_TUNE_CACHE``.
"""

import hashlib
import json
import os
import time

import numpy as np

from . import (ptsbe_plan, ptsbe_plan_compile, ptsbe_run_batch, ptsbe_trajset_from_records,
               ptsbe_workspace_size)


def candidates_for(n, precision):
    """(tile_qubits, min_fill, half_tile, pair_fusion) candidates: the two largest
    register-kernel tiles that fit n qubits (0 = the planner's choice when none
    does), fill 2 or 3, whole or half-tile register changes, pair fusion on or
    off.  13-qubit tiles (complex64) are left out: they measured slower on every
    size tried; name them with `candidates` to try them."""
    top = 12 if precision == "c64" else 11
    tiles = [t for t in range(top, 5, -1) if t <= n][:2] or [0]
    return [(t, f, h, pf) for t in tiles for f in (2, 3) for h in (False, True) for pf in (True, False)]


def autotune(circuit, precision="c64", records=None, sample=64, candidates=None, reps=2, params=None,
             stream=None, log=None):
    """Pick (tile_qubits, min_fill, half_tile, pair_fusion) for `circuit`.
    `records`: trajectory records (list of (site, k) tuples) to time on, e.g.
    from ts.get()["records"]; the first `sample` are used (an error-free record
    if none are given).  Returns {"tile_qubits", "min_fill", "half_tile",
    "pair_fusion", "results": [(tile, fill, half, pair, ms in the tile passes for
    the sample, compile s)], "seconds"}; the first four are ptsbe_plan's keyword
    arguments."""
    import torch
    t_start = time.perf_counter()
    n = circuit["n_qubits"]
    recs = list(records[:sample]) if records else [()]
    m = [1] * len(recs)
    cands = candidates or candidates_for(n, precision)
    results = []
    best = None
    obs = [(1.0, (0,))]
    for tile, fill, half, pair in cands:
        plan = ptsbe_plan(circuit, precision=precision, tile_qubits=tile, min_fill=fill, half_tile=half,
                          pair_fusion=pair)
        _, csec = ptsbe_plan_compile(plan)
        ts = ptsbe_trajset_from_records(plan, recs, m)
        ws = torch.empty(ptsbe_workspace_size(plan, ts, "expectation", params=params), dtype=torch.uint8,
                         device="cuda")
        out = {"expval": torch.empty(len(recs), dtype=torch.float64, device="cuda")}
        ptsbe_run_batch(plan, ts, mode="expectation", params=params, observable=obs, workspace=ws, out=out,
                        stream=stream)
        tms = []
        for _ in range(reps):
            tm = np.zeros(10)
            ptsbe_run_batch(plan, ts, mode="expectation", params=params, observable=obs, workspace=ws,
                            out=out, stream=stream, timing=tm)
            tms.append(tm[0])
        ms = float(min(tms))
        results.append((tile, fill, half, pair, ms, csec))
        if log:
            log(f"[tune] tile {tile} fill {fill} half-tile LDS {half} pair fusion {pair}: {ms:.3f} ms in "
                f"tile passes ({plan.info['n_passes']} passes), compile {csec:.1f} s")
        if best is None or ms < best[0]:
            best = (ms, tile, fill, half, pair)
        del ws, out
    return {"tile_qubits": best[1], "min_fill": best[2], "half_tile": best[3], "pair_fusion": best[4],
            "results": results, "seconds": time.perf_counter() - t_start}


DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def circuit_key(circuit, precision):
    """Cache key: SHA-256 of the circuit description (qubit count, ops, channels,
    rules, parameters) and the precision."""
    blob = json.dumps({"circuit": circuit, "precision": precision}, sort_keys=True,
                      default=lambda x: x.tolist() if hasattr(x, "tolist") else str(x))
    return hashlib.sha256(blob.encode()).hexdigest()[:32]


def _cache_path(path):
    return path or os.environ.get("PTSBE_TUNE_CACHE") or DEFAULT_CACHE


def load_cache(path=None):
    path = _cache_path(path)
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def tuned_plan_options(circuit, precision="c64", cache=None, tune_if_missing=False, retune=False, **kw):
    """ptsbe_plan keyword arguments for `circuit` from the tuning cache, tuning
    (and storing the pick) on a miss if `tune_if_missing`, else None on a miss;
    `retune` tunes and replaces the entry even on a hit.
    Returns (options or None, cache entry or None)."""
    cands = kw.get("candidates") or candidates_for(circuit["n_qubits"], precision)
    kw["candidates"] = cands
    key = circuit_key(circuit, precision)
    path = _cache_path(cache)
    entries = load_cache(path)
    e = None if retune else entries.get(key)
    if e is None and (tune_if_missing or retune):
        r = autotune(circuit, precision=precision, **kw)
        e = {"n_qubits": circuit["n_qubits"], "precision": precision,
             "pick": {k: r[k] for k in ("tile_qubits", "min_fill", "half_tile", "pair_fusion")},
             "results": [list(x) for x in r["results"]], "seconds": r["seconds"],
             "candidates": [list(c) for c in cands]}
        entries[key] = e
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(entries, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    if e is None:
        return None, None
    return dict(e["pick"]), e


def main(argv=None):
    """Tune the benchmark workloads and store the picks in the cache."""
    import argparse
    import sys
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c4", choices=["c2", "c4"])
    ap.add_argument("--cache", default=None)
    ap.add_argument("--sample", type=int, default=0, help="trajectories timed per candidate (0: by state size)")
    ap.add_argument("--candidates", default=None,
                    help="comma-separated tile:fill or tile:fill:h (h: half-tile register changes) entries, "
                         "pair fusion on; default: the full candidate set")
    ap.add_argument("--retune", action="store_true", help="tune again even where the cache has a pick")
    a = ap.parse_args(argv)
    cands = None
    if a.candidates:
        cands = []
        for c in a.candidates.split(","):
            f = c.split(":")
            cands.append((int(f[0]), int(f[1]), len(f) > 2 and f[2] == "h", True))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from workloads import c2_workload, c4_workload
    from . import ptsbe_sample_kraus
    wls = [c2_workload()] if a.workload == "c2" else [c4_workload(n) for n in (24, 26, 28)]

    def log(msg):
        sys.stderr.write(msg + "\n")
        sys.stderr.flush()

    for wl in wls:
        circ = wl["circuit"]
        n = circ["n_qubits"]
        plan = ptsbe_plan(circ, precision=wl["precision"], compile=False)
        pts = wl["pts"]
        ts = ptsbe_sample_kraus(plan, "proportional", n_draws=pts["n_draws"], total_shots=pts["total_shots"],
                                seed=wl["seed"], cfg=wl["cfg"])
        state = (8 if wl["precision"] == "c64" else 16) << n
        sample = a.sample or int(max(1, min(64, (8 << 30) // state)))
        opts, e = tuned_plan_options(circ, wl["precision"], cache=a.cache, tune_if_missing=True, retune=a.retune,
                                     records=ts.get()["records"], sample=sample, log=log, candidates=cands)
        log(f"[tune] {n} qubits: {opts} ({e['seconds']:.0f} s)")


if __name__ == "__main__":
    main()
