"""PTSBE throughput on one MI355X.

Workload (default): 20 qubits, 40 brick layers of random U3 + CZ with a coherent
RZ(eps) over-rotation per CZ, 1q depolarizing 1e-3 and 2q depolarizing 5e-3;
512 proportional pre-sampled draws sharing 10^6 shots (about 480 unique
trajectories), complex64 states with FP64 norms and CDFs.

One step = one ptsbe_run_batch call over the whole trajectory set: state
preparation of every trajectory (fused tile passes), FP64 norm + CDF scans,
and the sorted-uniform sampler writing 10^6 tagged shots -- inputs (plan
tables) resident, outputs left on the device.

Printed JSON: value = shots/s of batched PTSBE; the per-shot trajectory
baseline (Algorithm 1: one state preparation per shot, same kernels, same
GPU), the roofline of the dominant kernel (the tile pass) from the library's
HIP-event stage timer, and the FP64 oracle timed on the host on a bounded sample.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shots/s batched PTSBE vs per-shot trajectories; gate-kernel HBM GB/s"
HBM_PEAK_GBS = 8000.0
# FP32 vector peak of MI355X: 256 CUs x 2.4 GHz x 256 FLOP/clk/CU
FP32_PEAK_TFLOPS = 157.3
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "tile_pass_c2_traffic.md")


def log(msg):
    sys.stderr.write(msg + "\n")
    sys.stderr.flush()


_CPU_JOB = None     # (circuit, expanded steps, site channels, records, shots each, seed, cfg) for workers


def _oracle_worker_init():
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)


def _oracle_trajectory(i):
    """One trajectory of the oracle: state preparation + sampling (one thread)."""
    from oracle.sampling import sample
    from oracle.statevector import run_record
    circ, ss, ch, records, m, seed, cfg = _CPU_JOB
    psi, _ = run_record(circ, records[i], steps_sites=ss, chans=ch)
    sample(psi, m, seed, cfg, i)
    return i


def cpu_baseline(wl, g, budget_s=12.0, workers=16):
    """The oracle (complex128 NumPy) on the trajectory set, state preparation +
    sampling of the average shot count per trajectory, extrapolated linearly to
    whole-job shots/s: first on one thread for ``budget_s`` seconds (at least one
    trajectory), then trajectory-parallel over min(workers, host cores) processes
    (one thread each), one trajectory per process.  Call it before the process
    touches the GPU: the pool forks."""
    global _CPU_JOB
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.noise import expand, site_channels
    circ = wl["circuit"]
    avg_m = int(round(float(np.mean(g["m"]))))
    _CPU_JOB = (circ, expand(circ), site_channels(circ), g["records"], avg_m, wl["seed"], wl["cfg"])
    B = len(g["m"])
    done = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while done < B and (done == 0 or time.perf_counter() - t0 < budget_s):
            _oracle_trajectory(done)
            done += 1
        dt1 = time.perf_counter() - t0
    single = done * avg_m / dt1
    procs = max(1, min(workers, os.cpu_count() or 1))
    n_par = min(B, procs)
    with mp.get_context("fork").Pool(procs, initializer=_oracle_worker_init) as pool:
        t0 = time.perf_counter()
        for _ in pool.imap_unordered(_oracle_trajectory, range(n_par)):
            pass
        dtp = time.perf_counter() - t0
    par = n_par * avg_m / dtp
    _CPU_JOB = None
    return {"value": par, "unit": "shots/s", "cores": procs, "kind": "oracle",
            "sample": f"{n_par} of {B} trajectories prepared by the complex128 oracle, trajectory-parallel "
                      f"over {procs} processes of one thread, each sampled at the average {avg_m} shots "
                      f"({dtp:.1f} s), extrapolated linearly to the whole job",
            "single_thread": {"value": single, "unit": "shots/s", "cores": 1,
                              "sample": f"{done} trajectories on one thread ({dt1:.1f} s)"}}


def measured_traffic(plan):
    """HBM bytes per tile-pass dispatch from the committed counter summary, or
    None when the plan's kernels have changed since the counters were taken."""
    from paper_2504_16297_amd.profile_summary import kernel_fingerprint, read_traffic
    r = read_traffic(TRAFFIC_SUMMARY)
    if r is None or r[1] != kernel_fingerprint(plan):
        return None
    return r[0]


def pass_roofline(flops_per_launch, bytes_per_launch, launch_ms, traffic):
    """Roofline entry of the tile-pass kernels.  Their arithmetic intensity
    (useful FP32 flops per algorithmic HBM byte) against the machine balance
    (FP32 peak / HBM peak) decides which roof bounds them; the other roof is
    reported beside it."""
    tflops = flops_per_launch / (launch_ms * 1e-3) / 1e12
    gbs = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    ai = flops_per_launch / bytes_per_launch
    balance = FP32_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    hbm = {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    alu = {"achieved": tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tflops / FP32_PEAK_TFLOPS}
    main_roof, other = ("hbm", alu) if ai < balance else ("alu", hbm)
    r = {"bound": main_roof}
    r.update(hbm if main_roof == "hbm" else alu)
    r.update({"traffic": traffic, "kernel": "ptsbe_pass_* (compiled fused tile passes)",
              "avg_launch_ms": launch_ms, "flops_per_launch": flops_per_launch,
              "bytes_per_launch": bytes_per_launch, "flops_per_byte": ai, "machine_balance": balance,
              ("alu" if main_roof == "hbm" else "hbm"): other})
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-baseline", action="store_true", help="skip the per-shot GPU baseline")
    ap.add_argument("--baseline-shots", type=int, default=512)
    ap.add_argument("--fingerprint", action="store_true",
                    help="only print the kernel fingerprint of the 20-qubit workload's plan (host only)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 2 GiB device copy (calibrates FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5"],
                    help="c2: the 20-qubit headline workload; c3: the surface-code job (10^9 shots); "
                         "c4: the 24/26/28-qubit mixed batch and the "
                         "33- and 35-qubit trajectories; c5: the adjoint gradient of the 16-qubit ansatz")
    args = ap.parse_args()
    if args.fingerprint:
        import paper_2504_16297_amd as P
        from paper_2504_16297_amd.profile_summary import kernel_fingerprint
        from workloads import c2_workload
        wl = c2_workload()
        print(kernel_fingerprint(P.ptsbe_plan(wl["circuit"], precision=wl["precision"])))
        return
    if args.copy_probe:
        import torch
        n = 1 << 28                      # 2^28 float64 = 2 GiB read + 2 GiB written per copy
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the PTSBE path here is single-GPU (inter-trajectory "
              f"sharding is a partition of the trajectory set, not built); --gpus {args.gpus} is "
              f"not supported", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c4":
        return bench_c4(args)
    if args.workload == "c5":
        return bench_c5(args)
    if args.workload == "c3":
        return bench_c3(args)

    import numpy as np
    import torch

    import paper_2504_16297_amd as P
    from workloads import c2_workload

    wl = c2_workload()
    circ = wl["circuit"]
    pts = wl["pts"]
    t0 = time.perf_counter()
    plan = P.ptsbe_plan(circ, precision=wl["precision"])
    t_plan = time.perf_counter() - t0
    t0 = time.perf_counter()
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=pts["n_draws"], total_shots=pts["total_shots"],
                              seed=wl["seed"], cfg=wl["cfg"])
    t_pts = time.perf_counter() - t0
    g = ts.get()
    cpu = None
    if not args.no_cpu:
        # host-only so far (planning and PTS make no device calls): the oracle's
        # worker pool forks before the GPU is initialised
        log("[bench] timing the oracle on the host ...")
        cpu = cpu_baseline(wl, g)
        log(f"[bench] oracle {cpu['value']:.4g} shots/s on {cpu['cores']} processes, "
            f"{cpu['single_thread']['value']:.4g} on one thread")
    torch.cuda.set_device(0)
    B = len(g["m"])
    S = int(g["total_shots"])
    n_kernels, t_compile = P.ptsbe_plan_compile(plan)
    log(f"[bench] {wl['name']}: {B} unique trajectories, {plan.info['n_passes']} tile passes "
        f"({n_kernels} compiled kernels, {t_compile:.1f} s), plan {t_plan*1e3:.1f} ms, PTS {t_pts*1e3:.1f} ms")

    ws_bytes = P.ptsbe_workspace_size(plan, ts, mode="shots")
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out = {"bits": torch.empty(S, dtype=torch.int32, device="cuda"),
           "traj": torch.empty(S, dtype=torch.int32, device="cuda")}
    stream = torch.cuda.current_stream()

    def step(timing=None):
        return P.ptsbe_run_batch(plan, ts, mode="shots", seed=wl["seed"], cfg=wl["cfg"], workspace=ws,
                                 out=out, stream=stream, timing=timing)

    for i in range(args.warmup):
        step()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    timings = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        tm = np.zeros(10)
        step(tm)
        timings.append(tm)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    value = S * args.steps / dt
    T = np.sum(timings, axis=0)
    pass_ms = T[0] / T[1]
    pass_bytes = T[6] / T[1]
    pass_flops = T[8] / T[1]
    log(f"[bench] {ms_per_step:.2f} ms/step, {value:.4g} shots/s; passes {T[0]/args.steps:.2f} ms/step "
        f"({T[1]/args.steps:.0f} launches), scan {T[3]/args.steps:.2f} ms, sampler {T[4]/args.steps:.2f} ms")

    result = {"metric": METRIC, "value": value, "unit": "shots/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "c64 (fp32 state, fp64 norm/CDF)", "data": "synthetic",
              "config": {"workload": wl["name"], "n_qubits": 20, "layers": 40, "draws": pts["n_draws"],
                         "unique_trajectories": B, "total_shots": S, "parallelism": "single GPU, batched"},
              "roofline": pass_roofline(pass_flops, pass_bytes, pass_ms, measured_traffic(plan)),
              "stages_ms_per_step": {"passes": T[0] / args.steps, "scan": T[3] / args.steps,
                                     "sampler": T[4] / args.steps, "total_events": T[5] / args.steps},
              "state_passes_per_step": T[9] / args.steps, "state_passes_unshared": B * plan.info["n_passes"],
              "plan_ms": t_plan * 1e3, "pts_ms": t_pts * 1e3, "compile_s": t_compile,
              "compiled_kernels": n_kernels}

    # distinct shots of the last step (Fig. 4's unique fraction), outside the timed steps
    uws = torch.empty(P.ptsbe_unique_workspace_size(ts), dtype=torch.uint8, device="cuda")
    P.ptsbe_unique_shots(ts, out["bits"], workspace=uws, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = P.ptsbe_unique_shots(ts, out["bits"], workspace=uws, pairs=True, stream=stream)
    torch.cuda.synchronize()
    dt_u = time.perf_counter() - t0
    uniq = u["unique"].cpu().numpy().astype(np.float64)
    mm = np.asarray(g["m"], dtype=np.float64)
    result["distinct_shots"] = {"unique_fraction_of_all_shots": float(uniq.sum() / max(mm.sum(), 1.0)),
                                "mean_unique_fraction_per_trajectory": float(np.mean(uniq[mm > 0] / mm[mm > 0])),
                                "ms": dt_u * 1e3, "with_pairs": True}
    log(f"[bench] distinct shots: {uniq.sum() / mm.sum():.3f} of all shots are distinct within their "
        f"trajectory ({dt_u * 1e3:.2f} ms with (index, count) pairs)")
    del uws, u

    if not args.no_baseline:
        nb = args.baseline_shots
        tb = P.ptsbe_sample_kraus(plan, "per_shot", n_draws=nb, seed=wl["seed"], cfg=wl["cfg"])
        bws = torch.empty(P.ptsbe_workspace_size(plan, tb, mode="shots"), dtype=torch.uint8, device="cuda")
        bout = {"bits": torch.empty(nb, dtype=torch.int32, device="cuda"),
                "traj": torch.empty(nb, dtype=torch.int32, device="cuda")}
        P.ptsbe_run_batch(plan, tb, seed=wl["seed"], cfg=wl["cfg"], workspace=bws, out=bout)
        torch.cuda.synchronize()
        reps = 2
        t0 = time.perf_counter()
        for _ in range(reps):
            P.ptsbe_run_batch(plan, tb, seed=wl["seed"], cfg=wl["cfg"], workspace=bws, out=bout)
        torch.cuda.synchronize()
        bdt = time.perf_counter() - t0
        base = nb * reps / bdt
        result["per_shot_baseline"] = {"value": base, "unit": "shots/s",
                                       "shots": nb * reps, "seconds": bdt,
                                       "note": "Algorithm 1: one fresh draw and one full state "
                                               "preparation per shot, batched, same kernels"}
        result["speedup_vs_per_shot"] = value / base
        log(f"[bench] per-shot baseline {base:.4g} shots/s, speedup {value / base:.1f}x")
        del bws

    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result))


def bench_c4(args):
    """The mixed-size batch: brick circuits of 24, 26 and 28 qubits (30 layers,
    p2 = 1e-2) with 256 / 64 / 16 proportional draws x 10^5 shots, run back to
    back as one step; the per-shot baseline at 28 qubits; then one 33-qubit and
    one 35-qubit trajectory x 10^6 shots (64 and 256 GiB states), each timed on
    its own (the 35-qubit one only where the device has the memory)."""
    import numpy as np
    import torch

    import paper_2504_16297_amd as P
    from workloads import c4_workload

    torch.cuda.set_device(0)
    runs = []
    for n in (24, 26, 28):
        wl = c4_workload(n)
        pts = wl["pts"]
        plan = P.ptsbe_plan(wl["circuit"], precision="c64")
        ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=pts["n_draws"], total_shots=pts["total_shots"],
                                  seed=wl["seed"], cfg=wl["cfg"])
        nk, csec = P.ptsbe_plan_compile(plan)
        S = int(ts.get()["total_shots"])
        ws = torch.empty(P.ptsbe_workspace_size(plan, ts, mode="shots"), dtype=torch.uint8, device="cuda")
        out = {"bits": torch.empty(S, dtype=torch.int32, device="cuda"),
               "traj": torch.empty(S, dtype=torch.int32, device="cuda")}
        runs.append({"n": n, "wl": wl, "plan": plan, "ts": ts, "ws": ws, "out": out, "S": S})
        log(f"[bench c4] {n} qubits: {ts.n_traj} trajectories, {plan.info['n_passes']} passes, {nk} kernels "
            f"({csec:.1f} s), workspace {ws.numel() / 2**30:.1f} GiB")

    def step(timings=None):
        for i, r in enumerate(runs):
            tm = np.zeros(10) if timings is not None else None
            P.ptsbe_run_batch(r["plan"], r["ts"], seed=r["wl"]["seed"], cfg=r["wl"]["cfg"], workspace=r["ws"],
                              out=r["out"], timing=tm)
            if timings is not None:
                timings.append(tm)

    for i in range(args.warmup):
        step()
        log(f"[bench c4] warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    timings = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(timings)
        log(f"[bench c4] step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    S = sum(r["S"] for r in runs)
    value = S * args.steps / dt
    T = np.sum(timings, axis=0)
    per28 = np.sum(timings[2::3], axis=0)
    rate28 = runs[2]["S"] * args.steps / (per28[5] * 1e-3)
    pass_ms = T[0] / T[1]
    result = {"metric": METRIC, "value": value, "unit": "shots/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "dtype": "c64 (fp32 state, fp64 norm/CDF)",
              "data": "synthetic",
              "config": {"workload": "C4 mixed batch: 24/26/28 qubits x 30 brick layers, 256/64/16 draws "
                                     "x 1e5 shots", "total_shots": S,
                         "trajectories": [r["ts"].n_traj for r in runs], "parallelism": "single GPU, batched"},
              "roofline": pass_roofline(T[8] / T[1], T[6] / T[1], pass_ms, None),
              "q28_batched_shots_per_s": rate28}
    if not args.no_baseline:
        r = runs[2]
        nb = 8
        tb = P.ptsbe_sample_kraus(r["plan"], "per_shot", n_draws=nb, seed=r["wl"]["seed"], cfg=r["wl"]["cfg"])
        for x in runs:
            del x["ws"]
        torch.cuda.empty_cache()
        bws = torch.empty(P.ptsbe_workspace_size(r["plan"], tb, mode="shots"), dtype=torch.uint8, device="cuda")
        bout = {"bits": torch.empty(nb, dtype=torch.int32, device="cuda"),
                "traj": torch.empty(nb, dtype=torch.int32, device="cuda")}
        P.ptsbe_run_batch(r["plan"], tb, workspace=bws, out=bout)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.ptsbe_run_batch(r["plan"], tb, workspace=bws, out=bout)
        torch.cuda.synchronize()
        base = nb / (time.perf_counter() - t0)
        result["q28_per_shot_baseline_shots_per_s"] = base
        result["q28_speedup_vs_per_shot"] = rate28 / base
        log(f"[bench c4] 28 qubits: batched {rate28:.4g} shots/s, per-shot {base:.4g} shots/s, "
            f"speedup {rate28 / base:.1f}x")
        del bws
    runs.clear()
    torch.cuda.empty_cache()
    for nq in (33, 35):
        wl = c4_workload(nq)
        plan = P.ptsbe_plan(wl["circuit"], precision="c64")
        ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=1, total_shots=10**6, seed=wl["seed"],
                                  cfg=wl["cfg"])
        need = P.ptsbe_workspace_size(plan, ts, mode="shots")
        if torch.cuda.mem_get_info()[0] < need + (1 << 30):
            log(f"[bench c4] {nq} qubits: not enough device memory ({need / 2**30:.1f} GiB needed), skipped")
            continue
        P.ptsbe_plan_compile(plan)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        out = {"bits": torch.empty(10**6, dtype=torch.int64, device="cuda"),
               "traj": torch.empty(10**6, dtype=torch.int32, device="cuda")}
        P.ptsbe_run_batch(plan, ts, seed=wl["seed"], cfg=wl["cfg"], workspace=ws, out=out)
        torch.cuda.synchronize()
        log(f"[bench c4] {nq} qubits: warm-up run done")
        tm = np.zeros(10)
        t0 = time.perf_counter()
        P.ptsbe_run_batch(plan, ts, seed=wl["seed"], cfg=wl["cfg"], workspace=ws, out=out, timing=tm)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        result[f"q{nq}"] = {"shots": 10**6, "seconds": dt, "shots_per_s": 10**6 / dt,
                            "passes": plan.info["n_passes"], "pass_ms": tm[0], "state_gib": (1 << nq) * 8 / 2**30,
                            "pass_hbm_gbs": tm[6] / (tm[0] * 1e-3) / 1e9}
        log(f"[bench c4] {nq} qubits: {dt:.2f} s for 1e6 shots ({plan.info['n_passes']} passes, "
            f"{tm[6] / (tm[0] * 1e-3) / 1e9:.0f} GB/s in the passes)")
        del ws, out
        torch.cuda.empty_cache()
    print(json.dumps(result))


def bench_c3(args):
    """The surface-code memory experiment: 17 qubits (9 data + 8 ancilla), 5
    rounds with measure-resets, the 4096 most likely Kraus combinations sharing
    10^9 shots (reweighted allocation), every shot tagged with its trajectory;
    one step = plan tables uploaded, all trajectories prepared (measure-reset
    records decided on the device) and all 10^9 shots drawn into device buffers."""
    import numpy as np
    import torch

    import paper_2504_16297_amd as P
    from workloads import c3_workload

    torch.cuda.set_device(0)
    wl = c3_workload()
    pts = wl["pts"]
    plan = P.ptsbe_plan(wl["circuit"], precision=wl["precision"])
    t0 = time.perf_counter()
    ts = P.ptsbe_sample_kraus(plan, "most_likely", k_max=pts["k_max"], total_shots=pts["total_shots"],
                              seed=wl["seed"], cfg=wl["cfg"])
    t_pts = time.perf_counter() - t0
    g = ts.get()
    S = int(g["total_shots"])
    B = len(g["m"])
    n_kernels, t_compile = P.ptsbe_plan_compile(plan)
    ws = torch.empty(P.ptsbe_workspace_size(plan, ts, mode="shots"), dtype=torch.uint8, device="cuda")
    out = {"bits": torch.empty(S, dtype=torch.int32, device="cuda"),
           "traj": torch.empty(S, dtype=torch.int32, device="cuda"),
           "mr_bits": torch.empty(max(1, B * plan.info["n_measure"]), dtype=torch.uint8, device="cuda")}
    stream = torch.cuda.current_stream()
    log(f"[bench c3] {B} trajectories, {S} shots, {plan.info['n_passes']} passes, covered probability "
        f"{float(np.sum(g['p'])):.4f}, PTS {t_pts:.2f} s")

    def step(timing=None):
        P.ptsbe_run_batch(plan, ts, mode="shots", seed=wl["seed"], cfg=wl["cfg"], workspace=ws, out=out,
                          stream=stream, timing=timing)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench c3] warmup {i + 1}/{args.warmup} done")
    timings = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        tm = np.zeros(10)
        step(tm)
        timings.append(tm)
        log(f"[bench c3] step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    T = np.sum(timings, axis=0)
    value = S * args.steps / dt
    sampler_gbs = S * 8 * args.steps / (T[4] * 1e-3) / 1e9
    result = {"metric": "shots/s of the surface-code job (10^9 shots with trajectory tags)", "value": value,
              "unit": "shots/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "c64 (fp32 state, fp64 CDF)", "data": "synthetic",
              "config": {"workload": wl["name"], "trajectories": B, "total_shots": S},
              "stages_ms_per_step": {"passes": T[0] / args.steps, "measure_reset": T[2] / args.steps,
                                     "scan": T[3] / args.steps, "sampler": T[4] / args.steps},
              "sampler_output_gbs": sampler_gbs, "pts_s": t_pts, "compile_s": t_compile,
              "compiled_kernels": n_kernels}
    log(f"[bench c3] {dt * 1e3 / args.steps:.1f} ms/step, {value:.4g} shots/s; sampler "
        f"{T[4] / args.steps:.1f} ms ({sampler_gbs:.0f} GB/s of shot words and tags)")
    print(json.dumps(result))


def bench_c5(args):
    """Adjoint gradient of sum_i Z_i Z_(i+1) over the 16-qubit, 8-layer ansatz
    (256 parameters) with 1024 proportional draws: one step = E and all 256
    derivatives (forward preparation, lambda = O psi, reverse sweep, FP64
    reductions) for every trajectory; against that, the parameter-shift rule on
    the same GPU (2 expectation runs per parameter, timed on 8 parameters)."""
    import numpy as np
    import torch

    import paper_2504_16297_amd as P
    from workloads import c5_workload

    torch.cuda.set_device(0)
    wl = c5_workload()
    circ, obs = wl["circuit"], wl["observable"]
    params = np.asarray(circ["params"])
    pts = wl["pts"]
    plan = P.ptsbe_plan(circ, precision=wl["precision"])
    ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=pts["n_draws"], total_shots=pts["total_shots"],
                              seed=wl["seed"], cfg=wl["cfg"])
    P.ptsbe_plan_compile(plan)
    ws = torch.empty(P.ptsbe_workspace_size(plan, ts, "adjoint", params=params), dtype=torch.uint8, device="cuda")
    for _ in range(args.warmup):
        P.ptsbe_adjoint_grad(plan, ts, params, obs, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        E, G = P.ptsbe_adjoint_grad(plan, ts, params, obs, workspace=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ews = torch.empty(P.ptsbe_workspace_size(plan, ts, "expectation", params=params), dtype=torch.uint8,
                      device="cuda")
    out = {"expval": torch.empty(ts.n_traj, dtype=torch.float64, device="cuda")}
    P.ptsbe_run_batch(plan, ts, mode="expectation", params=params, observable=obs, workspace=ews, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(8):
        for sgn in (1.0, -1.0):
            pv = params.copy()
            pv[i] += sgn * np.pi / 2
            P.ptsbe_run_batch(plan, ts, mode="expectation", params=pv, observable=obs, workspace=ews, out=out)
    torch.cuda.synchronize()
    shift = (time.perf_counter() - t0) / 8 * params.size
    result = {"metric": "adjoint gradient evaluations/s (E and all derivatives over the trajectory set)",
              "value": 1.0 / dt, "unit": "gradients/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
              "dtype": "c64 (fp32 state, fp64 dots)", "data": "synthetic",
              "config": {"workload": wl["name"], "parameters": int(params.size), "trajectories": ts.n_traj},
              "E": float(E.cpu()[0]), "parameter_shift_seconds_estimate": shift,
              "speedup_vs_parameter_shift": shift / dt}
    log(f"[bench c5] {dt * 1e3:.1f} ms per gradient ({ts.n_traj} trajectories, {params.size} parameters); "
        f"parameter shift would take {shift:.2f} s")
    print(json.dumps(result))


if __name__ == "__main__":
    main()
