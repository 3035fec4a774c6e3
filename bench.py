"""PTSBE throughput on one MI355X.

Workload (default): the mixed-size batch -- brick circuits of 24, 26 and 28
qubits, 30 layers of random U3 + CZ with 2-qubit depolarizing noise
p2 = 1e-2 after every CZ, 256 / 64 / 16 proportional pre-sampled draws x 10^5
shots each (3.36e7 shots), complex64 states with FP64 norms and CDFs; plus one
33-qubit trajectory (64 GiB state) x 10^6 shots, reported beside it.

One step = one ptsbe_run_batch call per qubit count over its whole trajectory
set: state preparation of every trajectory (fused tile passes), FP64 norm +
CDF scans, and the sorted-uniform sampler writing every tagged shot -- plan
tables resident, outputs left on the device.

Printed JSON: value = shots/s of batched PTSBE over the whole batch; the
per-shot trajectory baseline at 28 qubits (Algorithm 1: one draw and one full
state preparation per shot, same kernels, same GPU, prefix sharing off), the
roofline of the dominant kernel (the tile passes) from the library's HIP-event
stage timer, the errors of one 24-qubit trajectory against the FP64 oracle,
and the oracle itself timed on the host on a bounded sample.
Other workloads: --workload c2 (20 qubits), c3 (surface code), c5 (gradient).
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
# FP32 vector peak of MI355X: 256 CUs x 2.4 GHz x 256 FLOP/clk/CU counts packed
# FP32 (two FMAs per lane and instruction).  The kernels here are built without
# packed FP32, so their ALU roof is half of it: 256 CUs x 4 SIMDs x 16 lanes x
# 2 FLOP (one FMA) x 2.4 GHz = 78.6 TFLOP/s (bench.py --rate-probe measures it).
FP32_PEAK_TFLOPS_PACKED = 157.3
FP32_PEAK_TFLOPS = 78.6
TRAFFIC_SUMMARY = {"c2": os.path.join(ROOT, "profiles", "tile_pass_c2_traffic.md"),
                   "c4": os.path.join(ROOT, "profiles", "tile_pass_c4_traffic.md")}
GOLDEN_C4 = os.path.join(ROOT, "tests", "golden", "c4_24q_trajectory.npz")
C4_SIZES = (24, 26, 28)


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


def host_info():
    """Host the oracle is timed on: logical CPUs, CPU model, RAM."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ram = None
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model, "ram_gib": ram}


_C4_JOB = None      # (circuit, expanded steps, site channels, records, ops per sample, shots, seed, cfg)


def _oracle_prefix(i, budget_s=None):
    """Trajectory i's preparation by the oracle, step by step: its first k
    steps (k from the job), or as many as fit ``budget_s`` seconds; then the
    sampling of m shots from that state (one thread).  Returns (k, preparation
    seconds, sampling seconds)."""
    import numpy as np
    from oracle.gates import gate_matrix
    from oracle.sampling import sample
    from oracle.statevector import apply, zero_state
    circ, (steps, sites), chans, records, k, m, seed, cfg = _C4_JOB
    n = circ["n_qubits"]
    ks = dict(records[i])
    psi = zero_state(n)
    t0 = time.perf_counter()
    done = 0
    while done < len(steps):
        if budget_s is None and done >= k:
            break
        if budget_s is not None and done >= 8 and time.perf_counter() - t0 >= budget_s:
            break
        st = steps[done]
        if st[0] == "gate":
            psi = apply(psi, n, gate_matrix(st[1], st[3]), st[2])
        elif st[0] == "site":
            _, us = chans[sites[st[1]]["channel"]]
            psi = apply(psi, n, us[ks.get(st[1], 0)], st[2])
        else:
            raise ValueError(st[0])
        done += 1
    t1 = time.perf_counter()
    psi = psi / np.linalg.norm(psi)
    sample(psi, m, seed, cfg, i)
    return done, t1 - t0, time.perf_counter() - t1


def _oracle_prefix_k(i):
    return _oracle_prefix(i)


def cpu_baseline_c4(budget_s=15.0, workers=16):
    """The oracle (complex128 NumPy) timed on a bounded sample of the mixed
    batch: a 24-qubit trajectory's preparation step by step for about
    ``budget_s`` seconds on one thread (its first k steps), then the sampling
    of 10^5 shots from that state; then the same sample trajectory-parallel,
    one thread per process, over min(workers, host CPUs) processes (the first
    k steps of one trajectory each).  Whole-job shots/s is extrapolated: a
    trajectory's preparation scales with its step count and 2^n, its sampling
    with 2^n (26 and 28 qubits: x4 and x16 per step).  Call it before the
    process touches the GPU: the pool forks."""
    global _C4_JOB
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits
    from oracle.noise import expand, site_channels, site_probs
    from oracle.pts import sample_kraus
    from workloads import c4_workload

    wls = {n: c4_workload(n) for n in C4_SIZES}
    wl = wls[24]
    circ = wl["circuit"]
    ss = expand(circ)
    ref = sample_kraus(site_probs(circ), wl["pts"], wl["seed"], wl["cfg"])
    m = int(round(sum(ref["m"]) / len(ref["m"])))
    n_steps24 = len(ss[0])
    _C4_JOB = (circ, ss, site_channels(circ), ref["records"], 0, m, wl["seed"], wl["cfg"])
    with threadpool_limits(limits=1):
        k, prep1, samp1 = _oracle_prefix(0, budget_s)
    _C4_JOB = _C4_JOB[:4] + (k,) + _C4_JOB[5:]
    procs = max(1, min(workers, os.cpu_count() or 1))
    with mp.get_context("fork").Pool(procs, initializer=_oracle_worker_init) as pool:
        t0 = time.perf_counter()
        res = list(pool.imap_unordered(_oracle_prefix_k, range(procs)))
        dtp = time.perf_counter() - t0
    _C4_JOB = None
    per_step = prep1 / k                       # seconds per 24-qubit step, one thread
    job1 = 0.0
    shots = 0
    for nq, w in wls.items():
        scale = 2.0 ** (nq - 24)
        n_steps = len(expand(w["circuit"])[0])
        job1 += w["pts"]["n_draws"] * (per_step * scale * n_steps + samp1 * scale)
        shots += w["pts"]["total_shots"]
    eff = (dtp / procs) / (prep1 + samp1)      # per-trajectory time when all processes run at once
    jobp = job1 * eff
    return {"value": shots / jobp, "unit": "shots/s", "cores": procs, "kind": "oracle",
            "sample": f"24-qubit trajectories: {k} of {n_steps24} preparation steps plus the sampling of {m} "
                      f"shots, one trajectory per process on {procs} processes of one thread ({dtp:.1f} s); "
                      f"extrapolated to the whole 24/26/28-qubit job by step count and 2^n (x4, x16)",
            "extrapolated": True,
            "single_thread": {"value": shots / job1, "unit": "shots/s", "cores": 1,
                              "sample": f"{k} steps of one 24-qubit trajectory ({prep1:.1f} s) and the sampling "
                                        f"of {m} shots ({samp1:.2f} s) on one thread, extrapolated likewise"},
            "host": host_info()}


def measured_traffic(plans, which):
    """HBM bytes per tile-pass dispatch from the committed counter summary, or
    None when the plans' kernels have changed since the counters were taken."""
    from paper_2504_16297_amd.profile_summary import read_traffic
    r = read_traffic(TRAFFIC_SUMMARY[which])
    if r is None or r[1] != fingerprint(plans):
        return None
    return r[0]


def fingerprint(plans):
    """Kernel fingerprint of one plan, or of several plans run in sequence."""
    import hashlib
    from paper_2504_16297_amd.profile_summary import kernel_fingerprint
    if not isinstance(plans, (list, tuple)):
        return kernel_fingerprint(plans)
    h = hashlib.sha256()
    for p in plans:
        h.update(kernel_fingerprint(p).encode())
    return h.hexdigest()[:16]


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


RATE_PROBE_SRC = r"""
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef float float16_t __attribute__((ext_vector_type(16)));
// FP32 FMA on the vector ALU: 8 independent chains per thread
extern "C" __global__ __launch_bounds__(256) void probe_valu_fma(float* out, int iters, float b, float c) {
  float a[8];
  for (int k = 0; k < 8; ++k) a[k] = (float)(threadIdx.x + k);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = __builtin_fmaf(a[k], b, c);
  }
  float s = 0.f;
  for (int k = 0; k < 8; ++k) s += a[k];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
// FP32 MFMA 16x16x4: 4 independent accumulators per wavefront
extern "C" __global__ __launch_bounds__(256) void probe_mfma_16x16x4(float* out, int iters, float b, float c) {
  float4_t acc[4];
  for (int k = 0; k < 4; ++k) acc[k] = (float4_t){c, c, c, c};
  const float x = (float)threadIdx.x * b;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, b, acc[k], 0, 0, 0);
  }
  float s = 0.f;
  for (int k = 0; k < 4; ++k) s += acc[k].x + acc[k].y + acc[k].z + acc[k].w;
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
// FP32 MFMA 32x32x2: 2 independent accumulators per wavefront
extern "C" __global__ __launch_bounds__(256) void probe_mfma_32x32x2(float* out, int iters, float b, float c) {
  float16_t acc[2];
  for (int k = 0; k < 2; ++k)
    for (int e = 0; e < 16; ++e) acc[k][e] = c;
  const float x = (float)threadIdx.x * b;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 2; ++k) acc[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(x, b, acc[k], 0, 0, 0);
  }
  float s = 0.f;
  for (int k = 0; k < 2; ++k)
    for (int e = 0; e < 16; ++e) s += acc[k][e];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
"""


def rate_probe():
    """FP32 issue rates of this GPU for the choice between the vector ALU and
    the matrix cores (MFMA) in the gate kernels: a kernel of independent
    v_fma_f32 chains and kernels of back-to-back FP32 MFMA (16x16x4, 32x32x2),
    compiled here with hiprtc, each launched over 4096 workgroups of 256
    threads and timed with events on torch's stream; prints one JSON line."""
    import ctypes as C

    import torch
    torch.cuda.set_device(0)
    rtc = C.CDLL("libhiprtc.so")
    hip = C.CDLL("libamdhip64.so")
    prog = C.c_void_p()
    if rtc.hiprtcCreateProgram(C.byref(prog), RATE_PROBE_SRC.encode(), b"rate_probe.hip", 0, None, None) != 0:
        raise SystemExit("hiprtcCreateProgram failed")
    opts = [b"--offload-arch=gfx950", b"-O3", b"-std=c++17", b"-Xclang", b"-target-feature", b"-Xclang",
            b"-packed-fp32-ops"]
    if rtc.hiprtcCompileProgram(prog, len(opts), (C.c_char_p * len(opts))(*opts)) != 0:
        n = C.c_size_t()
        rtc.hiprtcGetProgramLogSize(prog, C.byref(n))
        buf = C.create_string_buffer(n.value + 1)
        rtc.hiprtcGetProgramLog(prog, buf)
        raise SystemExit("rate probe does not compile:\n" + buf.value.decode(errors="replace"))
    n = C.c_size_t()
    rtc.hiprtcGetCodeSize(prog, C.byref(n))
    code = C.create_string_buffer(n.value)
    rtc.hiprtcGetCode(prog, code)
    mod = C.c_void_p()
    if hip.hipModuleLoadData(C.byref(mod), code) != 0:
        raise SystemExit("hipModuleLoadData failed")
    blocks, threads = 4096, 256
    out = torch.empty(blocks * threads, dtype=torch.float32, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    # (iterations, flops per launch): 8 chains x 2 flops per lane and iteration;
    # MFMA 2*M*N*K per wavefront instruction, 4 (16x16x4) or 2 (32x32x2) per
    # iteration; each launch about 50 ms
    waves = blocks * threads // 64
    kernels = {"probe_valu_fma": (512, 2 * 8 * 512 * blocks * threads),
               "probe_mfma_16x16x4": (64, 2 * 16 * 16 * 4 * 4 * 64 * waves),
               "probe_mfma_32x32x2": (64, 2 * 32 * 32 * 2 * 2 * 64 * waves)}
    res = {}
    for name, (iters, flops) in kernels.items():
        fn = C.c_void_p()
        if hip.hipModuleGetFunction(C.byref(fn), mod, name.encode()) != 0:
            raise SystemExit(f"no kernel {name}")
        a_out = C.c_void_p(out.data_ptr())
        a_it, a_b, a_c = C.c_int(iters), C.c_float(0.999), C.c_float(1e-3)
        params = (C.c_void_p * 4)(C.cast(C.byref(a_out), C.c_void_p), C.cast(C.byref(a_it), C.c_void_p),
                                  C.cast(C.byref(a_b), C.c_void_p), C.cast(C.byref(a_c), C.c_void_p))

        def launch():
            if hip.hipModuleLaunchKernel(fn, blocks, 1, 1, threads, 1, 1, 0, stream, params, None) != 0:
                raise SystemExit(f"launch of {name} failed")

        launch()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            launch()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / 5
        res[name] = {"ms": ms, "iterations": iters, "tflops": flops / (ms * 1e-3) / 1e12}
        log(f"[rate probe] {name}: {res[name]['tflops']:.1f} TFLOP/s ({ms:.3f} ms)")
    print(json.dumps({"rate_probe": res, "fp32_vector_peak_tflops_unpacked": FP32_PEAK_TFLOPS,
                      "fp32_vector_peak_tflops_packed": FP32_PEAK_TFLOPS_PACKED,
                      "launch": {"blocks": blocks, "threads": threads}}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-baseline", action="store_true", help="skip the per-shot GPU baseline")
    ap.add_argument("--baseline-shots", type=int, default=512)
    ap.add_argument("--fingerprint", action="store_true",
                    help="only print the kernel fingerprint of the workload's plans (host only)")
    ap.add_argument("--no-q33", action="store_true", help="skip the 33-qubit trajectory (c4)")
    ap.add_argument("--no-graph", action="store_true", help="skip the captured-graph replay of the step (c4)")
    ap.add_argument("--q35", action="store_true", help="also time one 35-qubit trajectory (c4)")
    ap.add_argument("--no-errors", action="store_true",
                    help="skip the 24-qubit trajectory's comparison with the stored oracle values (c4)")
    ap.add_argument("--rate-probe", action="store_true",
                    help="only measure the FP32 rates of the vector ALU and of FP32 MFMA on this GPU")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 2 GiB device copy (calibrates FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--workload", default="c4", choices=["c2", "c3", "c4", "c5"],
                    help="c4 (default): the 24/26/28-qubit mixed batch and the 33-qubit trajectory; "
                         "c2: the 20-qubit workload; c3: the surface-code job (10^9 shots); "
                         "c5: the adjoint gradient of the 16-qubit ansatz")
    args = ap.parse_args()
    if args.fingerprint:
        import paper_2504_16297_amd as P
        from workloads import c2_workload, c4_workload
        if args.workload == "c2":
            wl = c2_workload()
            print(fingerprint(P.ptsbe_plan(wl["circuit"], precision=wl["precision"])))
        elif args.workload == "c4":
            print(fingerprint([c4_plan(P, c4_workload(n))[0] for n in C4_SIZES]))
        else:
            raise SystemExit("--fingerprint: c2 or c4")
        return
    if args.rate_probe:
        return rate_probe()
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
    return bench_c2(args)


def bench_c2(args):
    """The 20-qubit workload: 40 brick layers of random U3 + CZ with a coherent
    RZ(eps) over-rotation per CZ, 1q depolarizing 1e-3 and 2q depolarizing
    5e-3; 512 proportional draws (about 480 unique trajectories) sharing 10^6
    shots, complex64."""
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
              "roofline": pass_roofline(pass_flops, pass_bytes, pass_ms, measured_traffic(plan, "c2")),
              "stages_ms_per_step": {"passes": T[0] / args.steps, "scan": T[3] / args.steps,
                                     "sampler": T[4] / args.steps, "total_events": T[5] / args.steps},
              "state_passes_per_step": T[9] / args.steps, "state_passes_unshared": B * plan.info["n_passes"],
              "plan_ms": t_plan * 1e3, "pts_ms": t_pts * 1e3, "compile_s": t_compile,
              "compiled_kernels": n_kernels}

    cr = copy_rate(torch, gib=1)
    result["roofline"]["copy_gbs"] = cr
    result["roofline"]["frac_of_copy"] = result["roofline"]["achieved"] / cr if result["roofline"]["bound"] == "hbm" \
        else result["roofline"]["hbm"]["achieved"] / cr

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


def c4_oracle_errors(P, plan, ts, m, bits_out, wl):
    """Errors of one 24-qubit trajectory against the FP64 oracle (values stored
    by tests/golden/make_golden.py): amplitudes at the stored basis indices and
    the mass of every 4096-amplitude block (a states-mode run of that
    trajectory), its first shots of the timed run against the oracle's (equal
    except within 1e-6 of a CDF boundary), and the total-variation distance of
    all its shots over 1024 bins of about equal oracle probability beside the
    distance expected from sampling noise alone."""
    import numpy as np
    import torch
    if not os.path.exists(GOLDEN_C4):
        return None
    gold = np.load(GOLDEN_C4)
    alpha = int(gold["alpha"])
    off = int(np.sum(np.asarray(m[:alpha], dtype=np.int64)))
    ma = int(m[alpha])
    shots = bits_out[off:off + ma].cpu().numpy().astype(np.int64)
    k = gold["shots"].size
    bad = np.flatnonzero(shots[:k] != gold["shots"])
    unexcused = int(np.sum(gold["boundary_distance"][bad] >= 1e-6))
    edges = gold["bin_edges"]
    hist = np.bincount(np.searchsorted(edges, shots, side="right") - 1, minlength=edges.size - 1)
    mass = gold["bin_mass"]
    tvd = 0.5 * float(np.sum(np.abs(hist / ma - mass)))
    tvd_noise = 0.5 * float(np.sum(np.sqrt(2.0 * mass * (1.0 - mass) / (np.pi * ma))))
    one = ts.slice(alpha, alpha + 1)
    st = P.ptsbe_run_batch(plan, one, mode="states")
    torch.cuda.synchronize()
    psi = st["states"][0]
    amp = psi[torch.as_tensor(gold["amp_index"], device=psi.device)].cpu().numpy().astype(np.complex128)
    block = (psi.real.double() ** 2 + psi.imag.double() ** 2).reshape(-1, 4096).sum(dim=1).cpu().numpy()
    del st, psi
    torch.cuda.empty_cache()
    return {"trajectory": alpha, "errors_in_record": int(gold["rec_site"].size), "shots_of_trajectory": ma,
            "max_amp_err": float(np.max(np.abs(amp - gold["amp"]))), "amplitudes_checked": int(amp.size),
            "max_block_mass_err": float(np.max(np.abs(block - gold["block_prob"]))),
            "shots_compared": int(k), "shot_mismatches": int(bad.size),
            "shot_mismatches_away_from_cdf_boundary": unexcused,
            "shot_mismatches_farther_than_1e-8": int(np.sum(gold["boundary_distance"][bad] >= 1e-8)),
            "mean_cdf_gap": 2.0 ** -24,
            "histogram_tvd_1024_bins": tvd, "tvd_expected_from_sampling": tvd_noise}


def c4_plan(P, wl):
    """The plan of one mixed-batch size with the autotuner's cached pick of its
    launch shape (tune_cache.json; the planner's defaults on a miss)."""
    from paper_2504_16297_amd.tune import tuned_plan_options
    opts, _ = tuned_plan_options(wl["circuit"], wl["precision"])
    return P.ptsbe_plan(wl["circuit"], precision=wl["precision"], **(opts or {})), opts


def c4_graph_replay(P, torch, runs, steps):
    """The mixed batch's step as one captured HIP graph per size (every tile
    pass, scan and sampler launch of that size's run), replayed `steps` times
    back to back on one created stream after a warm replay, whose shots and
    tags are compared with the last eager step's."""
    s = torch.cuda.Stream()
    ref = [(r["out"]["bits"].clone(), r["out"]["traj"].clone()) for r in runs]
    caps = [P.ptsbe_run_batch(r["plan"], r["ts"], seed=r["wl"]["seed"], cfg=r["wl"]["cfg"], workspace=r["ws"],
                              out=r["out"], stream=s, capture=True) for r in runs]
    for c in caps:
        c["bits"].fill_(-1)
        c["traj"].fill_(-1)
    torch.cuda.synchronize()
    for c in caps:
        c["graph"].launch(stream=s)
    s.synchronize()
    same = all(torch.equal(c["bits"], b) and torch.equal(c["traj"], t) for c, (b, t) in zip(caps, ref))
    t0 = time.perf_counter()
    for _ in range(steps):
        for c in caps:
            c["graph"].launch(stream=s)
    s.synchronize()
    dt = (time.perf_counter() - t0) / steps
    S = sum(r["S"] for r in runs)
    del caps, ref
    return {"graphs": len(runs), "steps": steps, "ms_per_step": dt * 1e3, "shots_per_s": S / dt,
            "bit_identical": bool(same)}


def copy_rate(torch, gib=4, reps=5):
    """GB/s (bytes read + written) of torch's device-to-device copy of `gib` GiB
    on the current GPU: a plain streaming kernel that reads and writes every
    byte once, the practical HBM ceiling beside the 8 TB/s peak."""
    n = (gib << 30) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * n * 8 / (ms * 1e-3) / 1e9


def bench_c4(args):
    """The mixed-size batch: brick circuits of 24, 26 and 28 qubits (30 layers,
    p2 = 1e-2) with 256 / 64 / 16 proportional draws x 10^5 shots, one
    ptsbe_run_batch call per size per step; the per-shot baseline at 28
    qubits; one 33-qubit trajectory x 10^6 shots (and with --q35 one 35-qubit
    trajectory), each timed on its own."""
    import numpy as np

    import paper_2504_16297_amd as P
    from workloads import c4_workload

    # The oracle is timed first, before this process makes any HIP call (the
    # pass compiler initialises the runtime), since its worker pool forks.
    cpu = None
    if not args.no_cpu:
        log("[bench c4] timing the oracle on the host ...")
        cpu = cpu_baseline_c4()
        log(f"[bench c4] oracle {cpu['value']:.4g} shots/s on {cpu['cores']} processes, "
            f"{cpu['single_thread']['value']:.4g} on one thread (extrapolated)")
    runs = []
    for n in C4_SIZES:
        wl = c4_workload(n)
        pts = wl["pts"]
        t0 = time.perf_counter()
        plan, opts = c4_plan(P, wl)
        ts = P.ptsbe_sample_kraus(plan, "proportional", n_draws=pts["n_draws"], total_shots=pts["total_shots"],
                                  seed=wl["seed"], cfg=wl["cfg"])
        t_host = time.perf_counter() - t0
        nk, csec = P.ptsbe_plan_compile(plan)
        g = ts.get()
        runs.append({"n": n, "wl": wl, "plan": plan, "ts": ts, "m": g["m"], "S": int(g["total_shots"]),
                     "host_ms": t_host * 1e3, "compile_s": csec, "kernels": nk, "tuned": opts})
        log(f"[bench c4] {n} qubits: {ts.n_traj} trajectories, {plan.info['n_passes']} passes, {nk} kernels "
            f"({csec:.1f} s), plan + PTS {t_host * 1e3:.0f} ms")
    plans = [r["plan"] for r in runs]

    import torch
    torch.cuda.set_device(0)
    for r in runs:
        r["ws"] = torch.empty(P.ptsbe_workspace_size(r["plan"], r["ts"], mode="shots"), dtype=torch.uint8,
                              device="cuda")
        r["out"] = {"bits": torch.empty(r["S"], dtype=torch.int32, device="cuda"),
                    "traj": torch.empty(r["S"], dtype=torch.int32, device="cuda")}
        log(f"[bench c4] {r['n']} qubits: workspace {r['ws'].numel() / 2**30:.1f} GiB")

    def step(timings=None):
        for r in runs:
            tm = np.zeros(10) if timings is not None else None
            P.ptsbe_run_batch(r["plan"], r["ts"], seed=r["wl"]["seed"], cfg=r["wl"]["cfg"], workspace=r["ws"],
                              out=r["out"], timing=tm)
            if timings is not None:
                timings.append(tm)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
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
    per_n = {r["n"]: np.sum(timings[i::len(runs)], axis=0) for i, r in enumerate(runs)}
    rate28 = runs[-1]["S"] * args.steps / (per_n[28][5] * 1e-3)
    pass_ms = T[0] / T[1]
    result = {"metric": METRIC, "value": value, "unit": "shots/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "dtype": "c64 (fp32 state, fp64 norm/CDF)",
              "data": "synthetic",
              "config": {"workload": "mixed-size batch: 24/26/28-qubit brick circuits x 30 layers (random U3 + CZ, "
                                     "2q depolarizing 1e-2), 256/64/16 proportional draws x 1e5 shots",
                         "total_shots": S, "trajectories": [r["ts"].n_traj for r in runs],
                         "parallelism": "single GPU, batched",
                         "plan_options": {str(r["n"]): r["tuned"] or "default (no cached tuning)" for r in runs}},
              "roofline": pass_roofline(T[8] / T[1], T[6] / T[1], pass_ms, measured_traffic(plans, "c4")),
              "stages_ms_per_step": {"passes": T[0] / args.steps, "scan": T[3] / args.steps,
                                     "sampler": T[4] / args.steps, "total_events": T[5] / args.steps},
              "per_size": {str(r["n"]): {"trajectories": r["ts"].n_traj, "passes": r["plan"].info["n_passes"],
                                         "ms_per_step": per_n[r["n"]][5] / args.steps,
                                         "pass_hbm_gbs": per_n[r["n"]][6] / (per_n[r["n"]][0] * 1e-3) / 1e9,
                                         "shots_per_s": r["S"] * args.steps / (per_n[r["n"]][5] * 1e-3)}
                           for r in runs},
              "compile_s": sum(r["compile_s"] for r in runs),
              "host_plan_pts_ms": sum(r["host_ms"] for r in runs)}
    rl = result["roofline"]
    log(f"[bench c4] {dt * 1e3 / args.steps:.1f} ms/step, {value:.4g} shots/s; passes {T[0] / args.steps:.1f} ms "
        f"({T[1] / args.steps:.0f} launches, {rl['bound']}-bound: {rl['achieved']:.1f} {rl['unit']}, "
        f"{rl['frac']:.3f} of {rl['peak']})")
    err = None
    if not args.no_errors:
        err = c4_oracle_errors(P, runs[0]["plan"], runs[0]["ts"], runs[0]["m"], runs[0]["out"]["bits"],
                               runs[0]["wl"])
    if err is not None:
        result["oracle_errors_24q"] = err
        log(f"[bench c4] 24-qubit trajectory {err['trajectory']} vs oracle: max|amp err| {err['max_amp_err']:.2e}, "
            f"{err['shot_mismatches']} of {err['shots_compared']} shots differ "
            f"({err['shot_mismatches_away_from_cdf_boundary']} away from a boundary), "
            f"TVD {err['histogram_tvd_1024_bins']:.4f} (sampling noise {err['tvd_expected_from_sampling']:.4f})")
    if not args.no_graph:
        gr = c4_graph_replay(P, torch, runs, min(args.steps, 5))
        result["graph_replay"] = gr
        log(f"[bench c4] captured step: {gr['graphs']} HIP graphs replayed {gr['steps']} times, "
            f"{gr['ms_per_step']:.1f} ms/step, {gr['shots_per_s']:.4g} shots/s, shots equal to the eager run's: "
            f"{gr['bit_identical']}")
    for r in runs:
        del r["ws"], r["out"]
    torch.cuda.empty_cache()
    cr = copy_rate(torch)
    rl = result["roofline"]
    pass_gbs = rl["achieved"] if rl["bound"] == "hbm" else rl["hbm"]["achieved"]
    rl["copy_gbs"] = cr
    rl["frac_of_copy"] = pass_gbs / cr
    log(f"[bench c4] device copy {cr:.0f} GB/s: the passes move {pass_gbs:.0f} GB/s, {pass_gbs / cr:.3f} of it")
    if not args.no_baseline:
        r = runs[-1]
        nb = 24
        tb = P.ptsbe_sample_kraus(r["plan"], "per_shot", n_draws=nb, seed=r["wl"]["seed"], cfg=r["wl"]["cfg"])
        bws = torch.empty(P.ptsbe_workspace_size(r["plan"], tb, mode="shots", prefix_sharing=False),
                          dtype=torch.uint8, device="cuda")
        bout = {"bits": torch.empty(nb, dtype=torch.int32, device="cuda"),
                "traj": torch.empty(nb, dtype=torch.int32, device="cuda")}

        def base_run():
            P.ptsbe_run_batch(r["plan"], tb, seed=r["wl"]["seed"], cfg=r["wl"]["cfg"], workspace=bws, out=bout,
                              prefix_sharing=False)

        base_run()
        torch.cuda.synchronize()
        reps = 0
        t0 = time.perf_counter()
        while reps == 0 or time.perf_counter() - t0 < 1.0:
            base_run()
            torch.cuda.synchronize()
            reps += 1
        bdt = time.perf_counter() - t0
        base = nb * reps / bdt
        result["per_shot_baseline"] = {
            "value": base, "unit": "shots/s", "qubits": 28, "shots": nb * reps, "seconds": bdt,
            "note": "Algorithm 1 at 28 qubits: one fresh draw and one full state preparation per shot "
                    "(prefix sharing off), 24 shots per batch, same kernels and GPU"}
        result["q28_batched_shots_per_s"] = rate28
        result["speedup_vs_per_shot_q28"] = rate28 / base
        log(f"[bench c4] 28 qubits: batched {rate28:.4g} shots/s, per-shot {base:.4g} shots/s "
            f"({nb * reps} shots in {bdt:.2f} s), speedup {rate28 / base:.1f}x")
        del bws, bout
        torch.cuda.empty_cache()
    big = [] if args.no_q33 else [33]
    if args.q35:
        big.append(35)
    for nq in big:
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
        dtb = time.perf_counter() - t0
        result[f"q{nq}"] = {"shots": 10**6, "seconds": dtb, "shots_per_s": 10**6 / dtb,
                            "passes": plan.info["n_passes"], "pass_ms": tm[0], "state_gib": (1 << nq) * 8 / 2**30,
                            "pass_hbm_gbs": tm[6] / (tm[0] * 1e-3) / 1e9}
        log(f"[bench c4] {nq} qubits: {dtb:.2f} s for 1e6 shots ({plan.info['n_passes']} passes, "
            f"{tm[6] / (tm[0] * 1e-3) / 1e9:.0f} GB/s in the passes)")
        del ws, out
        torch.cuda.empty_cache()
    if cpu is not None:
        result["cpu_baseline"] = cpu
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
