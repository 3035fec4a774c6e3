"""Run the generated pass kernels on the CPU (test helper).

Each pass's generated HIP source (ptsbe_plan_pass_source) is compiled with g++
against a small shim: one OS thread per GPU thread of a block, __syncthreads as
a std::barrier, the block's LDS as a static buffer, HIP's bit-cast intrinsics
as memcpy.  The shim runs the kernel over the whole grid on the exported
device tables, so the pass compiler's output can be checked against the oracle
without a GPU.  Measure-reset steps between passes follow the same rule as the
table emulator.
"""

import ctypes as C
import hashlib
import os
import subprocess
import tempfile

import numpy as np

import paper_2504_16297_amd as P
from paper_2504_16297_amd import _lib as L
from paper_2504_16297_amd.tables import export_tables

SHIM = r"""
#include <cstdint>
#include <cstring>
#include <barrier>
#include <thread>
#include <vector>
struct float2 { float x, y; };
struct double2 { double x, y; };
struct uint2 { unsigned x, y; };
struct Dim3 { unsigned x = 0, y = 0, z = 0; };
thread_local Dim3 threadIdx, blockIdx;
Dim3 blockDim, gridDim;
static std::barrier<>* g_bar = nullptr;
static inline void __syncthreads() { g_bar->arrive_and_wait(); }
alignas(16) unsigned char smem[1 << 17];
static inline float __uint_as_float(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }
static inline uint32_t __float_as_uint(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }
static inline double __longlong_as_double(long long u) { double f; std::memcpy(&f, &u, 8); return f; }
static double g_shfl[1024];
// lane exchange within `width` lanes, by way of a block-wide buffer: every
// thread of the block calls it at the same point, as the kernels do
static inline double __shfl_xor(double v, int mask, int width) {
  g_shfl[threadIdx.x] = v;
  __syncthreads();
  const unsigned src = (threadIdx.x & ~(unsigned)(width - 1)) | ((threadIdx.x ^ mask) & (width - 1));
  const double r = g_shfl[src];
  __syncthreads();
  return r;
}
static inline long long __double_as_longlong(double f) { long long u; std::memcpy(&u, &f, 8); return u; }
static inline uint32_t atomicOr(uint32_t* p, uint32_t v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
// every lane of a wave reads the same LDS word after a barrier where the kernels call it
static inline uint32_t __builtin_amdgcn_readfirstlane(uint32_t v) { return v; }
#define __global__
#define __device__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define __shared__
#define __align__(x)
#define __builtin_nontemporal_load(p) (*(p))
#define __builtin_nontemporal_store(v, p) (*(p) = (v))
"""

RUNNER = r"""
extern "C" int run_pass(const unsigned char* blob, const uint64_t* offs, unsigned pass, unsigned slot_begin,
                        void* states, uint64_t N, unsigned n, unsigned k, unsigned n_passes, unsigned rows,
                        const uint8_t* mr_bits, const double* mr_norm, unsigned n_measure, void* lam,
                        double* partial, unsigned n_dot) {
  (void)lam; (void)partial; (void)n_dot;
  PassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.passes = blob + offs[0];
  a.ops = blob + offs[1];
  a.slot_default = reinterpret_cast<const uint32_t*>(blob + offs[2]) + slot_begin;
  a.pool = reinterpret_cast<const V*>(blob + offs[3]);
  a.ov_off = reinterpret_cast<const uint32_t*>(blob + offs[4]);
  a.ov = reinterpret_cast<const DOverride*>(blob + offs[5]);
  a.mr_bits = mr_bits;
  a.mr_norm = mr_norm;
  a.states = reinterpret_cast<V*>(states);
  a.route = nullptr;
  a.carrier0 = 0;
  a.N = N;
  a.n = n;
  a.pass = pass;
  a.n_passes = n_passes;
  a.t0 = 0;
  a.n_measure = n_measure;
  const unsigned bx = 1u << (k - 4), gx = (1u << (n - k)) / PASS_TPB;
  blockDim.x = bx;
  gridDim.x = gx;
  gridDim.y = rows;
  for (unsigned y = 0; y < rows; ++y)
    for (unsigned x = 0; x < gx; ++x) {
      std::barrier<> bar(bx);
      g_bar = &bar;
      std::vector<std::thread> th;
      for (unsigned t = 0; t < bx; ++t)
        th.emplace_back([&, t]() {
          threadIdx.x = t;
          blockIdx.x = x;
          blockIdx.y = y;
          ptsbe_pass(a PASS_EXTRA);
        });
      for (auto& h : th) h.join();
    }
  return 0;
}
"""

_CACHE = os.path.join(tempfile.gettempdir(), "ptsbe_compiled_cpu")


def pass_source(plan, p, adjoint=False):
    n = C.c_size_t()
    P.check(L.lib().ptsbe_plan_pass_source(plan.handle, p, int(adjoint), None, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    P.check(L.lib().ptsbe_plan_pass_source(plan.handle, p, int(adjoint), buf, C.byref(n)))
    return buf.value.decode()


def _build(src):
    os.makedirs(_CACHE, exist_ok=True)
    h = hashlib.sha256(src.encode()).hexdigest()[:20]
    so = os.path.join(_CACHE, h + ".so")
    if not os.path.exists(so):
        cpp = os.path.join(_CACHE, h + ".cpp")
        extra = "#define PASS_EXTRA , reinterpret_cast<V*>(lam), partial, n_dot\n" if "double* partial" in src \
            else "#define PASS_EXTRA\n"
        # two tiles per workgroup: half the grid
        extra += "#define PASS_TPB %du\n" % (2 if "tile_id0 = 2ull * blockIdx.x" in src else 1)
        with open(cpp, "w") as f:
            f.write(SHIM + src + extra + RUNNER)
        tmp = so + f".{os.getpid()}.tmp"
        r = subprocess.run(["g++", "-std=c++20", "-O1", "-fPIC", "-shared", "-pthread", "-w", cpp, "-o", tmp],
                           stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if r.returncode:
            raise RuntimeError("g++ failed on generated pass source:\n" + r.stdout[:4000])
        os.replace(tmp, so)
    lib = C.CDLL(so)
    lib.run_pass.restype = C.c_int
    lib.run_pass.argtypes = [C.c_void_p, C.c_void_p, C.c_uint, C.c_uint, C.c_void_p, C.c_uint64, C.c_uint,
                             C.c_uint, C.c_uint, C.c_uint, C.c_void_p, C.c_void_p, C.c_uint, C.c_void_p,
                             C.c_void_p, C.c_uint]
    return lib


def _raw_tables(ts, params):
    pa = None
    if params is not None and len(params):
        pa = np.ascontiguousarray(params, dtype=np.float64)
    pp = C.cast(pa.ctypes.data, C.POINTER(C.c_double)) if pa is not None else None
    n = C.c_size_t()
    offs = np.zeros(16, dtype=np.uint64)
    P.check(L.lib().ptsbe_trajset_tables(ts.handle, pp, 0, None, C.byref(n), offs.ctypes.data))
    buf = np.zeros(n.value, dtype=np.uint8)
    P.check(L.lib().ptsbe_trajset_tables(ts.handle, pp, 0, buf.ctypes.data, C.byref(n), offs.ctypes.data))
    return buf, offs


def _channel_decision(circuit, chan, gidx, p1, be, alpha):
    """The device's decision for a state-dependent channel entry (test side:
    the oracle's uniforms and channel definition)."""
    from oracle.channels import general_channel, kraus_ops
    from oracle.rng import key1, uniforms
    d0, d1 = general_channel(kraus_ops(circuit["channels"][chan]))
    probs = [d0[k] * (1.0 - p1) + d1[k] * p1 for k in range(len(d0))]
    u = uniforms(be[0], key1(4, be[1], alpha), gidx + 1)[gidx]
    c, last, k = 0.0, 0, None
    for kk, pp in enumerate(probs):
        c += pp
        if pp > 0.0:
            last = kk
            if k is None and u < c:
                k = kk
    k = last if k is None else k
    return k, probs[k]


# The library's storage layout of states above 2^12 amplitudes (PTSBE_PLAN_NO_SWIZZLE
# turns it off): amplitude x sits at x ^ (f(x >> 12) << 4), with f the XOR of the
# 8-bit constants below over the set bits of x >> 12.  An involution.
SWIZZLE = (0x7a, 0x96, 0x3d, 0x72, 0x37, 0xf0, 0x85, 0x96, 0x92, 0xce, 0x15, 0x7a,
           0xaf, 0xa8, 0x5d, 0x0e, 0xaa, 0x06, 0xed, 0x62, 0x47, 0x60, 0x35, 0x86)


def storage_positions(n, on=True):
    """Position of each amplitude x (0 .. 2^n - 1) in the library's state storage."""
    x = np.arange(1 << n, dtype=np.int64)
    if not on or n <= 12:
        return x
    h = x >> 12
    f = np.zeros_like(x)
    for i, c in enumerate(SWIZZLE):
        f ^= ((h >> i) & 1) * c
    return x ^ (f << 4)


def run_compiled(plan, ts, params=None, mr_tol=1e-6, circuit=None, be=(0, 0), swizzled=None):
    """States [B, 2^n] (normalised) after running every pass through its
    generated kernel on the CPU.  State-dependent channel entries are decided
    as the device does, with ``circuit``'s channels and ``be`` = (seed, cfg)."""
    info = plan.info
    n = info["n_qubits"]
    N = 1 << n
    B = ts.n_traj
    t = export_tables(ts, params)
    blob, offs = _raw_tables(ts, params)
    passes = t["passes"]
    NP = len(passes)
    c64 = info["precision"] == L.C64
    states = np.zeros((B, N), dtype=np.complex64 if c64 else np.complex128)
    nm = info["n_measure"]
    mr_bits = np.zeros(max(1, B * nm), dtype=np.uint8)
    mr_norm = np.zeros(max(1, B * nm), dtype=np.float64)
    slot_begin = [int(ps["slot_begin"]) for ps in passes]
    libs = {}
    x = np.arange(N, dtype=np.int64)
    if swizzled is None:
        swizzled = bool(info["swizzled"])
    pos = storage_positions(n, swizzled)     # amplitude x is states[:, pos[x]]
    for ex in t["exec"]:
        if ex["pass"] != 0xFFFFFFFF:
            p = int(ex["pass"])
            src = pass_source(plan, p)
            if not src:
                raise RuntimeError(f"pass {p} has no compiled kernel")
            if src not in libs:
                libs[src] = _build(src)
            k = int(passes[p]["k"])
            libs[src].run_pass(blob.ctypes.data, offs.ctypes.data, p, slot_begin[p], states.ctypes.data, N, n, k,
                               NP, B, mr_bits.ctypes.data, mr_norm.ctypes.data, nm, None, None, 0)
        else:
            rinfo = plan.record_info()
            for b in range(B):
                w = np.abs(states[b][pos].astype(np.complex128)) ** 2
                tot = w.sum()
                for j in range(int(ex["nq"])):
                    q = int(ex["q"][j])
                    p1 = w[((x >> q) & 1) == 1].sum() / tot
                    r = int(ex["idx"][j])
                    chan, gidx = rinfo[r]
                    if chan >= 0:
                        k, pk = _channel_decision(circuit, chan, gidx, p1, be, b)
                        mr_bits[b * nm + r] = k
                        mr_norm[b * nm + r] = 1.0 / np.sqrt(pk * tot) if j == 0 else 1.0 / np.sqrt(pk)
                        continue
                    if min(p1, 1 - p1) > mr_tol:
                        raise RuntimeError(f"non-deterministic measure-reset on qubit {q}")
                    bit = 1 if p1 > 0.5 else 0
                    pb = p1 if bit else 1 - p1
                    mr_bits[b * nm + r] = bit
                    mr_norm[b * nm + r] = 1.0 / np.sqrt(pb * tot) if j == 0 else 1.0 / np.sqrt(pb)
    out = states[:, pos].astype(np.complex128)
    return out / np.linalg.norm(out, axis=1, keepdims=True)


def run_compiled_adjoint(plan, ts, params, odiag):
    """(E, grad) of the trajectory set with the forward and reverse-sweep
    passes run through their generated kernels on the CPU: psi by the forward
    kernels, lambda = O psi, the dual-state sweep kernels writing one FP64
    partial per (trajectory, tile, wavefront, term), reduced with weights
    count / sum count."""
    from paper_2504_16297_amd.tables import export_adjoint_tables
    info = plan.info
    n, N, B = info["n_qubits"], 1 << info["n_qubits"], ts.n_traj
    c64 = info["precision"] == L.C64
    cdt = np.complex64 if c64 else np.complex128
    psi = run_compiled(plan, ts, params).astype(cdt)   # normalised: unitary circuits keep the norm
    lam = (psi.astype(np.complex128) * odiag[None, :]).astype(cdt)
    # into storage order (the layout the reverse-sweep kernels read)
    pos = storage_positions(n, bool(info["swizzled"]))
    psi_s = np.empty_like(psi)
    lam_s = np.empty_like(lam)
    psi_s[:, pos] = psi
    lam_s[:, pos] = lam
    psi, lam = np.ascontiguousarray(psi_s), np.ascontiguousarray(lam_s)
    adj, dot_param = export_adjoint_tables(ts, params)
    n_raw = C.c_size_t()
    offs = np.zeros(16, dtype=np.uint64)
    pa = np.ascontiguousarray(params, dtype=np.float64)
    pp = C.cast(pa.ctypes.data, C.POINTER(C.c_double))
    P.check(L.lib().ptsbe_trajset_adjoint_tables(ts.handle, pp, None, C.byref(n_raw), offs.ctypes.data, None, None))
    blob = np.zeros(n_raw.value, dtype=np.uint8)
    P.check(L.lib().ptsbe_trajset_adjoint_tables(ts.handle, pp, blob.ctypes.data, C.byref(n_raw), offs.ctypes.data,
                                                 None, None))
    passes = adj["passes"]
    NP = len(passes)
    n_dot = len(dot_param)
    k = int(passes[0]["k"])
    W = max(1, (1 << (k - 4)) // 64)
    tiles = (1 << (n - k)) * W
    partial = np.zeros(B * tiles * max(1, n_dot), dtype=np.float64)
    libs = {}
    for ex in adj["exec"]:
        p = int(ex["pass"])
        src = pass_source(plan, p, adjoint=True)
        if not src:
            raise RuntimeError(f"reverse-sweep pass {p} has no compiled kernel")
        if src not in libs:
            libs[src] = _build(src)
        libs[src].run_pass(blob.ctypes.data, offs.ctypes.data, p, int(passes[p]["slot_begin"]), psi.ctypes.data, N,
                           n, int(passes[p]["k"]), NP, B, None, None, 0, lam.ctypes.data, partial.ctypes.data, n_dot)
    g = ts.get()
    w = g["count"].astype(np.float64) / g["count"].sum()
    part = partial.reshape(B, tiles, max(1, n_dot))[:, :, :n_dot].sum(axis=1)
    grad = np.zeros(info["n_params"])
    for d in range(n_dot):
        grad[int(dot_param[d])] += float(np.dot(w, part[:, d]))
    fwd = run_compiled(plan, ts, params)
    E = float(np.dot(w, (np.abs(fwd) ** 2 * odiag[None, :]).sum(axis=1)))
    return E, grad
