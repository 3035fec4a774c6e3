// gfx950 kernels of the PTSBE hot path.
//
//  k_pass      one fused tile pass: a 2^k-amplitude tile (k tile qubits, the
//              lowest ones always included so that global accesses are runs of
//              >= 128 contiguous bytes) is staged in LDS, every fused 1- and
//              2-qubit operation of the pass is applied to it in order (with
//              the trajectory's own matrices for slots touched by its noise
//              record), and the tile is written back.  Grid: (tile, state).
//  k_marginal  FP64 partial sums of |psi|^2 restricted to x_q = 1 for a group
//              of measured qubits (general Kraus branch of Algorithm 1).
//  k_mr_decide per trajectory: outcome b = [p1 > 1/2], determinism check,
//              renormalisation factor.
//  k_mr_follow under prefix sharing: the prefix state's decisions copied to
//              the trajectories still on it.
//  k_blocksum / k_scan_partials / k_cdf
//              FP64 norm and inclusive prefix sum of |psi|^2 per state:
//              per-thread sequential sums, wavefront shuffles, an LDS tree,
//              then block offsets (reduce-then-scan, no inter-block waiting).
//  k_sample    per (trajectory, chunk of shots): Philox4x64-10 uniforms, a
//              bitonic sort (strides below 16 in registers, 16 elements per
//              thread), and an upper-bound search of u * total in the CDF,
//              each thread's next sorted element searched from its previous
//              result on; writes the basis index and the trajectory id of
//              each shot.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "philox.hpp"

namespace ptsbe {

template <typename V>
struct Real;
template <>
struct Real<float2> {
  using T = float;
};
template <>
struct Real<double2> {
  using T = double;
};

template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
  V r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

template <typename V>
__device__ __forceinline__ V cfma2(V m0, V x0, V m1, V x1) {
  V r;
  r.x = m0.x * x0.x - m0.y * x0.y + m1.x * x1.x - m1.y * x1.y;
  r.y = m0.x * x0.y + m0.y * x0.x + m1.x * x1.y + m1.y * x1.x;
  return r;
}

__device__ __forceinline__ uint64_t tile_offset(uint32_t L, const uint8_t* tq, uint32_t k) {
  uint64_t off = 0;
#pragma unroll
  for (int j = 0; j < kMaxTileBits; ++j)
    if (j < (int)k) off |= (uint64_t)((L >> j) & 1u) << tq[j];
  return off;
}

// Source / destination state slots of this block row, and whose overrides apply.
struct Route {
  uint32_t src, dst, t;
  bool carrier;
};
template <typename V>
__device__ __forceinline__ Route route_of(const PassArgs<V>& a) {
  Route r;
  r.src = r.dst = blockIdx.y;
  if (a.route) {
    const uint2 e = a.route[blockIdx.y];
    r.src = e.x;
    r.dst = e.y;
  }
  r.carrier = a.route != nullptr && r.dst >= a.carrier0;
  r.t = r.carrier ? a.carrier_t : a.t0 + r.dst;
  return r;
}

template <typename V>
__global__ __launch_bounds__(256) void k_pass(PassArgs<V> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const DPass& P = a.passes[a.pass];
  const uint32_t k = P.k;
  const uint32_t nt = 1u << k;
  V* tile = reinterpret_cast<V*>(smem);
  uint32_t* slot_off = reinterpret_cast<uint32_t*>(smem + sizeof(V) * nt);
  __shared__ uint8_t tq[16];
  const uint32_t tid = threadIdx.x;
  const Route rt = route_of(a);
  const uint32_t t = rt.t;                            // trajectory (set-local index)
  const uint64_t tile_id = blockIdx.x;
  if (tid < 16) tq[tid] = P.tq[tid];
  uint64_t base = 0;
  for (uint32_t i = 0; i < a.n - k; ++i)
    if ((tile_id >> i) & 1) base |= 1ull << P.oq[i];
  const V* sst = a.states + (uint64_t)rt.src * a.N;
  V* st = a.states + (uint64_t)rt.dst * a.N;
  for (uint32_t s = tid; s < P.n_slots; s += blockDim.x) slot_off[s] = a.slot_default[P.slot_begin + s];
  __syncthreads();
  if (!rt.carrier) {
    const uint32_t ob = a.ov_off[(uint64_t)t * a.n_passes + a.pass];
    const uint32_t oe = a.ov_off[(uint64_t)t * a.n_passes + a.pass + 1];
    for (uint32_t i = ob + tid; i < oe; i += blockDim.x) slot_off[a.ov[i].slot] = a.ov[i].off;
  }
  const bool init = (P.flags & PASS_INIT_ZERO) != 0;
  for (uint32_t L = tid; L < nt; L += blockDim.x) {
    V v;
    if (init) {
      v.x = (base == 0 && L == 0) ? 1 : 0;
      v.y = 0;
    } else {
      v = sst[swizzle(base + tile_offset(L, tq, k), a.swz)];
    }
    tile[L] = v;
  }
  __syncthreads();
  const DOp* ops = a.ops + P.op_begin;
  for (uint32_t o = 0; o < P.n_ops; ++o) {
    const DOp op = ops[o];
    if (op.type == DOP_M1) {
      const V* m = a.pool + slot_off[op.slot[0]];
      const V m00 = m[0], m01 = m[1], m10 = m[2], m11 = m[3];
      const uint32_t bit = 1u << op.a, lo = bit - 1;
      for (uint32_t pr = tid; pr < nt / 2; pr += blockDim.x) {
        const uint32_t i0 = ((pr & ~lo) << 1) | (pr & lo);
        const uint32_t i1 = i0 | bit;
        const V x0 = tile[i0], x1 = tile[i1];
        tile[i0] = cfma2(m00, x0, m01, x1);
        tile[i1] = cfma2(m10, x0, m11, x1);
      }
    } else if (op.type == DOP_M2) {
      const V* m = a.pool + slot_off[op.slot[0]];
      const uint32_t A = 1u << op.a, B = 1u << op.b;
      const uint32_t l1 = min(A, B) - 1, l2 = max(A, B) - 1;
      for (uint32_t qd = tid; qd < nt / 4; qd += blockDim.x) {
        uint32_t i = ((qd & ~l1) << 1) | (qd & l1);
        i = ((i & ~l2) << 1) | (i & l2);
        const uint32_t idx[4] = {i, i | A, i | B, i | A | B};
        V x[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = tile[idx[r]];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          V acc = cfma2(m[r * 4 + 0], x[0], m[r * 4 + 1], x[1]);
          V acc2 = cfma2(m[r * 4 + 2], x[2], m[r * 4 + 3], x[3]);
          acc.x += acc2.x;
          acc.y += acc2.y;
          tile[idx[r]] = acc;
        }
      }
    } else if (op.type == DOP_D1 || op.type == DOP_D2) {
      const V* m = a.pool + slot_off[op.slot[0]];
      const bool two = op.type == DOP_D2;
      const uint32_t dd = two ? 5 : 3;  // stride of the diagonal in a 4x4 / 2x2 row-major matrix
      const uint32_t fa = op.a == 255 ? (uint32_t)((base >> op.ga) & 1) : 0;
      const uint32_t fb = (two && op.b == 255) ? (uint32_t)((base >> op.gb) & 1) : 0;
      for (uint32_t L = tid; L < nt; L += blockDim.x) {
        uint32_t ba = op.a == 255 ? fa : (L >> op.a) & 1u;
        uint32_t bb = two ? (op.b == 255 ? fb : (L >> op.b) & 1u) : 0;
        const V ph = m[(ba + 2 * bb) * dd];
        tile[L] = cmul(ph, tile[L]);
      }
    } else if (op.type == DOP_DSIGN) {
      const uint32_t fa = op.a == 255 ? (uint32_t)((base >> op.ga) & 1) : 0;
      const uint32_t fb = op.b == 255 ? (uint32_t)((base >> op.gb) & 1) : 0;
      for (uint32_t L = tid; L < nt; L += blockDim.x) {
        const uint32_t ba = op.a == 255 ? fa : (L >> op.a) & 1u;
        const uint32_t bb = op.b == 254 ? 0u : (op.b == 255 ? fb : (L >> op.b) & 1u);
        if ((op.slot[0] >> (ba + 2 * bb)) & 1u) {
          V v = tile[L];
          v.x = -v.x;
          v.y = -v.y;
          tile[L] = v;
        }
      }
    } else if (op.type == DOP_KR) {
      // state-dependent channel: K_k / sqrt(p_k), k and the factor from the record
      const uint64_t ri = (uint64_t)t * a.n_measure + op.slot[0];
      const typename Real<V>::T sc = (typename Real<V>::T)a.mr_norm[ri];
      const V* m = a.pool + slot_off[op.slot[1]] + 4u * a.mr_bits[ri];
      V mm[4];
      for (int e = 0; e < 4; ++e) {
        mm[e] = m[e];
        mm[e].x *= sc;
        mm[e].y *= sc;
      }
      const uint32_t bit = 1u << op.a, lo = bit - 1;
      for (uint32_t pr = tid; pr < nt / 2; pr += blockDim.x) {
        const uint32_t i0 = ((pr & ~lo) << 1) | (pr & lo);
        const uint32_t i1 = i0 | bit;
        const V x0 = tile[i0], x1 = tile[i1];
        tile[i0] = cfma2(mm[0], x0, mm[1], x1);
        tile[i1] = cfma2(mm[2], x0, mm[3], x1);
      }
    } else if (op.type == DOP_MR) {
      const uint64_t ri = (uint64_t)t * a.n_measure + op.slot[0];
      const uint32_t b = a.mr_bits[ri];
      const typename Real<V>::T sc = (typename Real<V>::T)a.mr_norm[ri];
      const uint32_t bit = 1u << op.a, lo = bit - 1;
      for (uint32_t pr = tid; pr < nt / 2; pr += blockDim.x) {
        const uint32_t i0 = ((pr & ~lo) << 1) | (pr & lo);
        const uint32_t i1 = i0 | bit;
        V x = b ? tile[i1] : tile[i0];
        x.x *= sc;
        x.y *= sc;
        V z;
        z.x = 0;
        z.y = 0;
        tile[i0] = x;
        tile[i1] = z;
      }
    }
    __syncthreads();
  }
  for (uint32_t L = tid; L < nt; L += blockDim.x) st[swizzle(base + tile_offset(L, tq, k), a.swz)] = tile[L];
}

// ------------------------------------------------------- register tile pass
//
// Each thread keeps 16 amplitudes of the tile in registers; they span the 4
// local bits R (the "register bits"), the thread index supplies the other
// k - 4 local bits.  Gates on register bits are applied in registers with no
// data movement; a DOP_PHASE op changes R by writing the registers to LDS and
// reading them back in the new layout (XOR-swizzled to spread LDS banks).
// Loads and stores use R = the top 4 local bits, so the low local bits (the
// contiguous low qubits) run across lanes.

template <typename V>
struct Amp16 {
  V v[16];
};

template <int J, typename V>
__device__ __forceinline__ void reg_1q(Amp16<V>& s, V m00, V m01, V m10, V m11) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (r & (1 << J)) continue;
    const V x0 = s.v[r], x1 = s.v[r | (1 << J)];
    s.v[r] = cfma2(m00, x0, m01, x1);
    s.v[r | (1 << J)] = cfma2(m10, x0, m11, x1);
  }
}

template <typename V>
__device__ __forceinline__ V cdot4(const V* row, V x0, V x1, V x2, V x3) {
  V acc = cfma2(row[0], x0, row[1], x1);
  V acc2 = cfma2(row[2], x2, row[3], x3);
  acc.x += acc2.x;
  acc.y += acc2.y;
  return acc;
}

template <int J, typename V>
__device__ __forceinline__ void reg_1q_lds(Amp16<V>& s, const V* m) {
  // keep the matrix loads next to their use (hoisting them raises register pressure)
  asm volatile("" ::: "memory");
  const V m00 = m[0], m01 = m[1], m10 = m[2], m11 = m[3];
  reg_1q<J>(s, m00, m01, m10, m11);
}

template <int J, typename V>
__device__ __forceinline__ void reg_mr(Amp16<V>& s, uint32_t b, typename Real<V>::T sc) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (r & (1 << J)) continue;
    V x = b ? s.v[r | (1 << J)] : s.v[r];
    x.x *= sc;
    x.y *= sc;
    s.v[r] = x;
    s.v[r | (1 << J)].x = 0;
    s.v[r | (1 << J)].y = 0;
  }
}

// Negate the amplitudes whose bit r is set in `neg` by flipping IEEE sign bits.
__device__ __forceinline__ void reg_flip_signs(Amp16<float2>& s, uint32_t neg) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const uint32_t m = (neg << (31 - r)) & 0x80000000u;
    s.v[r].x = __uint_as_float(__float_as_uint(s.v[r].x) ^ m);
    s.v[r].y = __uint_as_float(__float_as_uint(s.v[r].y) ^ m);
  }
}

__device__ __forceinline__ void reg_flip_signs(Amp16<double2>& s, uint32_t neg) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const unsigned long long m = (unsigned long long)((neg >> r) & 1u) << 63;
    s.v[r].x = __longlong_as_double((long long)((unsigned long long)__double_as_longlong(s.v[r].x) ^ m));
    s.v[r].y = __longlong_as_double((long long)((unsigned long long)__double_as_longlong(s.v[r].y) ^ m));
  }
}

__device__ __forceinline__ uint32_t lds_swz(uint32_t L) { return L ^ ((L >> 4) & 15u); }

// Local index of register r given the thread part and the 4 register bit values.
__device__ __forceinline__ uint32_t reg_local(uint32_t Lt, const uint32_t* rb, int r) {
  return Lt | ((r & 1) ? rb[0] : 0) | ((r & 2) ? rb[1] : 0) | ((r & 4) ? rb[2] : 0) | ((r & 8) ? rb[3] : 0);
}

// Thread part of the local index: tid with zeros inserted at the register bits
// (ascending).
__device__ __forceinline__ uint32_t thread_local_part(uint32_t tid, const uint32_t* R) {
  uint32_t L = tid;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t lo = (1u << R[j]) - 1u;
    L = ((L & ~lo) << 1) | (L & lo);
  }
  return L;
}

// LDS of the register kernel: tile | first 4 entries of every slot matrix | ops | slot offsets.
template <typename V>
__host__ __device__ inline size_t reg_lds_bytes(uint32_t k, uint32_t n_slots, uint32_t n_ops) {
  return sizeof(V) * ((size_t(1) << k) + 4 * (size_t)n_slots) + sizeof(DOp) * (size_t)n_ops + 4 * (size_t)n_slots;
}

template <typename V>
__global__ __launch_bounds__(256) void k_pass_reg(PassArgs<V> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const DPass& P = a.passes[a.pass];
  const uint32_t k = P.k;
  const uint32_t n_slots = P.n_slots, n_ops = P.n_ops;
  V* tile = reinterpret_cast<V*>(smem);
  V* mats = tile + (size_t(1) << k);
  DOp* opl = reinterpret_cast<DOp*>(mats + 4 * (size_t)n_slots);
  uint32_t* slot_off = reinterpret_cast<uint32_t*>(opl + n_ops);
  const uint32_t tid = threadIdx.x;
  const Route rt = route_of(a);
  const uint32_t t = rt.t;
  const uint64_t tile_id = blockIdx.x;
  uint64_t base = 0;
  for (uint32_t i = 0; i < a.n - k; ++i)
    if ((tile_id >> i) & 1) base |= 1ull << P.oq[i];
  const V* sst = a.states + (uint64_t)rt.src * a.N;
  V* st = a.states + (uint64_t)rt.dst * a.N;
  for (uint32_t s = tid; s < n_slots; s += blockDim.x) slot_off[s] = a.slot_default[P.slot_begin + s];
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.ops + P.op_begin);
    uint32_t* dst = reinterpret_cast<uint32_t*>(opl);
    for (uint32_t i = tid; i < 4 * n_ops; i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  if (!rt.carrier) {
    const uint32_t ob = a.ov_off[(uint64_t)t * a.n_passes + a.pass];
    const uint32_t oe = a.ov_off[(uint64_t)t * a.n_passes + a.pass + 1];
    for (uint32_t i = ob + tid; i < oe; i += blockDim.x) slot_off[a.ov[i].slot] = a.ov[i].off;
  }
  __syncthreads();
  // every slot matrix has at least 4 entries; 1-qubit ops read theirs from LDS
  for (uint32_t i = tid; i < 4 * n_slots; i += blockDim.x) mats[i] = a.pool[slot_off[i >> 2] + (i & 3)];
  __syncthreads();

  // load layout: register bits = the top 4 local bits, thread index = the low k - 4 bits
  uint32_t R[4] = {k - 4, k - 3, k - 2, k - 1};
  uint32_t rb[4] = {1u << R[0], 1u << R[1], 1u << R[2], 1u << R[3]};
  uint32_t Lt = tid;
  const uint64_t ot = tile_offset(Lt, P.tq, k);
  uint64_t og[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) og[j] = 1ull << P.tq[R[j]];
  Amp16<V> s;
  const bool init = (P.flags & PASS_INIT_ZERO) != 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const uint64_t off = ot + ((r & 1) ? og[0] : 0) + ((r & 2) ? og[1] : 0) + ((r & 4) ? og[2] : 0) +
                         ((r & 8) ? og[3] : 0);
    if (init) {
      s.v[r].x = (base == 0 && Lt == 0 && r == 0) ? 1 : 0;
      s.v[r].y = 0;
    } else {
      s.v[r] = sst[swizzle(base + off, a.swz)];
    }
  }

  const DOp* ops = opl;
  uint32_t neg = 0;
  const uint32_t M[4] = {0xAAAAu, 0xCCCCu, 0xF0F0u, 0xFF00u};
  V cs;                 // pending block-uniform scalar (phases/signs of qubits outside the tile)
  cs.x = 1;
  cs.y = 0;
  bool pending = false;
  for (uint32_t o = 0; o < n_ops; ++o) {
    const DOp op = ops[o];
    const uint32_t type = op.type;
    if (type == DOP_M1G) {
      const uint32_t mk = op.mask;
      if (pending) {
        // the pending scalar rides on the group's first matrix: fold it into
        // that slot's LDS copy (every thread reads before anyone writes)
        const uint32_t s0 = (mk & 1u) ? op.slot[0] : (mk & 2u) ? op.slot[1] : (mk & 4u) ? op.slot[2] : op.slot[3];
        V* m = mats + 4u * s0;
        if (tid < 4) m[tid] = cmul(cs, m[tid]);
        __syncthreads();
        cs.x = 1;
        cs.y = 0;
        pending = false;
      }
      // all four positions, idle ones through the identity slot: one straight line
      reg_1q_lds<0>(s, mats + 4u * (uint32_t)op.slot[0]);
      reg_1q_lds<1>(s, mats + 4u * (uint32_t)op.slot[1]);
      reg_1q_lds<2>(s, mats + 4u * (uint32_t)op.slot[2]);
      reg_1q_lds<3>(s, mats + 4u * (uint32_t)op.slot[3]);
    } else if (type == DOP_M2) {
      // general 4x4 matrices go through the LDS tile (any two local bits)
      const uint32_t off = __builtin_amdgcn_readfirstlane(slot_off[op.slot[0]]);
      const V* m = a.pool + off;
#pragma unroll
      for (int r = 0; r < 16; ++r) tile[lds_swz(reg_local(Lt, rb, r))] = s.v[r];
      __syncthreads();
      const uint32_t A = 1u << op.a, B = 1u << op.b;
      const uint32_t l1 = min(A, B) - 1, l2 = max(A, B) - 1;
      const uint32_t nq4 = 1u << (k - 2);
      for (uint32_t qd = tid; qd < nq4; qd += blockDim.x) {
        uint32_t i = ((qd & ~l1) << 1) | (qd & l1);
        i = ((i & ~l2) << 1) | (i & l2);
        const uint32_t i0 = lds_swz(i), i1 = lds_swz(i | A), i2 = lds_swz(i | B), i3 = lds_swz(i | A | B);
        const V x0 = tile[i0], x1 = tile[i1], x2 = tile[i2], x3 = tile[i3];
        tile[i0] = cdot4(m, x0, x1, x2, x3);
        tile[i1] = cdot4(m + 4, x0, x1, x2, x3);
        tile[i2] = cdot4(m + 8, x0, x1, x2, x3);
        tile[i3] = cdot4(m + 12, x0, x1, x2, x3);
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) s.v[r] = tile[lds_swz(reg_local(Lt, rb, r))];
      __syncthreads();
    } else if (type == DOP_DSIGN) {
      uint32_t A1, B1, B0;
      if (op.a == 255) {
        A1 = ((base >> op.ga) & 1) ? 0xFFFFu : 0u;
      } else {
        const uint32_t la = op.a;
        A1 = la == R[0] ? M[0] : la == R[1] ? M[1] : la == R[2] ? M[2] : la == R[3] ? M[3]
                                                                    : (((Lt >> la) & 1) ? 0xFFFFu : 0u);
      }
      if (op.b == 254) {
        B1 = 0u;
      } else if (op.b == 255) {
        B1 = ((base >> op.gb) & 1) ? 0xFFFFu : 0u;
      } else {
        const uint32_t lb = op.b;
        B1 = lb == R[0] ? M[0] : lb == R[1] ? M[1] : lb == R[2] ? M[2] : lb == R[3] ? M[3]
                                                                    : (((Lt >> lb) & 1) ? 0xFFFFu : 0u);
      }
      const uint32_t A0 = ~A1 & 0xFFFFu;
      B0 = ~B1 & 0xFFFFu;
      const uint32_t mk = op.slot[0];
      neg ^= ((mk & 1) ? (A0 & B0) : 0u) | ((mk & 2) ? (A1 & B0) : 0u) | ((mk & 4) ? (A0 & B1) : 0u) |
             ((mk & 8) ? (A1 & B1) : 0u);
    } else if (type == DOP_SFLIP) {
      // neg may differ between threads (signs on thread bits), so it is applied
      // here and never folded into the block-uniform pending scalar
      reg_flip_signs(s, neg);
      neg = 0;
    } else if ((type == DOP_D1 && op.a == 255) || (type == DOP_D2 && op.a == 255 && op.b == 255)) {
      // diagonal on qubits outside the tile: one phase for the whole tile, folded
      // into the pending scalar (applied through the next 2x2 matrix or at the end)
      const V* m = mats + 4 * (uint32_t)op.slot[0];
      V ph;
      if (type == DOP_D1) {
        ph = ((base >> op.ga) & 1) ? m[3] : m[0];
      } else {
        const uint32_t i = (uint32_t)((base >> op.ga) & 1) + 2 * (uint32_t)((base >> op.gb) & 1);
        ph = a.pool[__builtin_amdgcn_readfirstlane(slot_off[op.slot[0]]) + 5 * i];
      }
      cs = cmul(cs, ph);
      pending = true;
    } else if (type == DOP_D1 || type == DOP_D2) {
      const uint32_t off = __builtin_amdgcn_readfirstlane(slot_off[op.slot[0]]);
      const V* m = a.pool + off;
      const bool two = type == DOP_D2;
      const uint32_t dd = two ? 5 : 3;
      const V d0 = m[0], d1 = m[dd], d2 = two ? m[2 * dd] : m[0], d3 = two ? m[3 * dd] : m[0];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint32_t L = reg_local(Lt, rb, r);
        const uint32_t ba = op.a == 255 ? (uint32_t)((base >> op.ga) & 1) : (L >> op.a) & 1u;
        const uint32_t bb = !two ? 0u : (op.b == 255 ? (uint32_t)((base >> op.gb) & 1) : (L >> op.b) & 1u);
        const uint32_t i = ba + 2 * bb;
        const V ph = i == 0 ? d0 : i == 1 ? d1 : i == 2 ? d2 : d3;
        s.v[r] = cmul(ph, s.v[r]);
      }
    } else if (type == DOP_MR) {
      const uint64_t ri = (uint64_t)t * a.n_measure + op.slot[0];
      const uint32_t b = a.mr_bits[ri];
      const typename Real<V>::T sc = (typename Real<V>::T)a.mr_norm[ri];
      const uint32_t la = op.a;
      if (la == R[0]) reg_mr<0>(s, b, sc);
      else if (la == R[1]) reg_mr<1>(s, b, sc);
      else if (la == R[2]) reg_mr<2>(s, b, sc);
      else reg_mr<3>(s, b, sc);
    } else if (type == DOP_KR) {
      const uint64_t ri = (uint64_t)t * a.n_measure + op.slot[0];
      const typename Real<V>::T sc = (typename Real<V>::T)a.mr_norm[ri];
      const V* m = a.pool + slot_off[op.slot[1]] + 4u * a.mr_bits[ri];
      V mm[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        mm[e] = m[e];
        mm[e].x *= sc;
        mm[e].y *= sc;
      }
      const uint32_t la = op.a;
      if (la == R[0]) reg_1q<0>(s, mm[0], mm[1], mm[2], mm[3]);
      else if (la == R[1]) reg_1q<1>(s, mm[0], mm[1], mm[2], mm[3]);
      else if (la == R[2]) reg_1q<2>(s, mm[0], mm[1], mm[2], mm[3]);
      else reg_1q<3>(s, mm[0], mm[1], mm[2], mm[3]);
    } else if (type == DOP_PHASE) {
#pragma unroll
      for (int r = 0; r < 16; ++r) tile[lds_swz(reg_local(Lt, rb, r))] = s.v[r];
      __syncthreads();
      R[0] = op.a;
      R[1] = op.b;
      R[2] = op.ga;
      R[3] = op.gb;
#pragma unroll
      for (int j = 0; j < 4; ++j) rb[j] = 1u << R[j];
      Lt = thread_local_part(tid, R);
#pragma unroll
      for (int r = 0; r < 16; ++r) s.v[r] = tile[lds_swz(reg_local(Lt, rb, r))];
      __syncthreads();
    }
  }
  if (pending) {
#pragma unroll
    for (int r = 0; r < 16; ++r) s.v[r] = cmul(cs, s.v[r]);
  }
  // the program ends in the load layout again
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const uint64_t off = ot + ((r & 1) ? og[0] : 0) + ((r & 2) ? og[1] : 0) + ((r & 4) ? og[2] : 0) +
                         ((r & 8) ? og[3] : 0);
    st[swizzle(base + off, a.swz)] = s.v[r];
  }
}

// ------------------------------------------------------------ FP64 reductions

__device__ __forceinline__ double wave_incl_scan(double v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    double o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive running maximum of `v` over the block's threads in thread order
// (`lo` for thread 0) and the block maximum.
__device__ __forceinline__ double block_excl_max(double v, double lo, double* total) {
  __shared__ double wmax[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const double o = __shfl_up(inc, d, 64);
    if (lane >= d) inc = fmax(inc, o);
  }
  double ex = __shfl_up(inc, 1, 64);
  if (lane == 0) ex = lo;
  if (lane == 63) wmax[w] = inc;
  __syncthreads();
  double before = lo, all = lo;
  for (int i = 0; i < 4; ++i) {
    if (i < w) before = fmax(before, wmax[i]);
    all = fmax(all, wmax[i]);
  }
  __syncthreads();
  *total = all;
  return fmax(before, ex);
}

// Exclusive prefix of `v` over the block (256 threads, fixed order) and the
// block total; identical arithmetic wherever it is called.
__device__ __forceinline__ void block_excl_scan(double v, double* excl, double* total) {
  __shared__ double wsum[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double inc = wave_incl_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  double woff = 0.0;
  for (int i = 0; i < w; ++i) woff += wsum[i];
  double tot = 0.0;
  for (int i = 0; i < 4; ++i) tot += wsum[i];
  *excl = woff + (inc - v);
  *total = tot;
  __syncthreads();
}

template <typename V>
__device__ __forceinline__ double norm2(V v) {
  return (double)v.x * (double)v.x + (double)v.y * (double)v.y;
}

// One block handles per_block (<= 4096) consecutive amplitudes of a state:
// |psi_x|^2 in FP64 is staged in LDS with coalesced loads (padded every 16
// entries), then each thread sums a contiguous run sequentially and the block
// combines the runs with wavefront shuffles and an LDS tree.  The block-sum
// and CDF kernels share this code, so a block's total is bit-identical in both
// and the CDF is monotone across block boundaries.
__device__ __forceinline__ uint32_t scan_pad(uint32_t e) { return e + (e >> 4); }

template <typename V, bool kWriteCdf>
__device__ __forceinline__ void block_prob_scan(const ScanArgs<V>& a) {
  __shared__ double sh[kScanBlock + kScanBlock / 16];
  const uint32_t b = blockIdx.x;
  V* st = a.states + (uint64_t)blockIdx.y * a.N;
  const uint64_t e0 = (uint64_t)b * a.per_block;
  const uint32_t E = a.per_block, per = a.per_thread, tid = threadIdx.x;
  // the block's amplitudes sit in its own 4096 positions, permuted by an XOR
  const uint32_t sx = E == kScanBlock ? swizzle_block(b, a.swz) : 0u;
  if (E == kScanBlock) {
    // full block: all 16 loads of a thread in flight before the first use
    constexpr uint32_t kPer = kScanBlock / 256;
    double w[kPer];
#pragma unroll
    for (uint32_t i = 0; i < kPer; ++i) w[i] = norm2(st[e0 + ((tid + 256u * i) ^ sx)]);
#pragma unroll
    for (uint32_t i = 0; i < kPer; ++i) sh[scan_pad(tid + 256u * i)] = w[i];
  } else {
    for (uint32_t e = tid; e < E; e += blockDim.x) sh[scan_pad(e)] = norm2(st[e0 + e]);
  }
  __syncthreads();
  const bool active = tid * per < E;
  double v[16];
  double s = 0.0;
  if (active)
    for (uint32_t i = 0; i < per; ++i) {
      s += sh[scan_pad(tid * per + i)];
      v[i] = s;
    }
  double ex, tot;
  block_excl_scan(s, &ex, &tot);   // ends with a barrier
  const uint64_t yb = (uint64_t)blockIdx.y * a.nblk + b;
  // Monotone CDF.  Element e = tid * per + i gets off + A_e with A_e = ex + v[i];
  // A is non-decreasing within a thread but rounding can make it dip by an ulp
  // where one thread's run meets the next, and off + A where one block meets the
  // next.  With a.maxa set, each CDF entry is the running maximum of those
  // values over all earlier entries (blocks: floor[b], the largest value of the
  // blocks before b), so every upper-bound search on it returns the first entry
  // above its argument.  The counting kernel writes each block's largest A.
  const bool mono = a.maxa != nullptr;
  double thr_floor = 0.0;
  if (mono) {
    const double top = active ? ex + v[per - 1] : 0.0;
    double bmax;
    if (!kWriteCdf) {
      block_excl_max(top, 0.0, &bmax);
      if (tid == 0) a.maxa[yb] = bmax;
    } else {
      const double off0 = a.offs[yb];
      thr_floor = block_excl_max(active ? off0 + top : 0.0, a.floor[yb], &bmax);
    }
  }
  // Support lists.  The CDF entry of element e = tid * per + i is off + A_e with
  // A_e = ex + v[i]; since adding off is monotone, an upper-bound search can
  // only return the block's first element or an element whose A exceeds the
  // previous element's.  Those elements (a superset of the possible results)
  // form the list; the counting and the writing kernels compute the same A.
  const bool support = a.sup_part != nullptr;
  uint32_t nz = 0;  // bit i: element tid * per + i is in the list
  double sex = 0.0, stot = 0.0;
  if (support) {
    __shared__ double last_a[256];
    if (active) last_a[tid] = ex + v[per - 1];
    __syncthreads();
    if (active) {
      double prev = tid == 0 ? 0.0 : last_a[tid - 1];
      for (uint32_t i = 0; i < per; ++i) {
        const double A = ex + v[i];
        if ((tid == 0 && i == 0) || A > prev) nz |= 1u << i;
        prev = A;
      }
    }
    block_excl_scan((double)__popc(nz), &sex, &stot);
  }
  if (!kWriteCdf) {
    if (tid == 0) {
      a.partial[yb] = tot;
      if (support) a.sup_part[yb] = stot;
    }
    return;
  }
  const double off = a.offs[yb];
  if (active)
    for (uint32_t i = 0; i < per; ++i) {
      const double c = off + (ex + v[i]);
      v[i] = mono ? fmax(thr_floor, c) : c;
      sh[scan_pad(tid * per + i)] = v[i];
    }
  if (support && active && a.sup_count[blockIdx.y] <= kSupportMax) {
    // the state's support list: its nonzero entries with their CDF values, in index order
    uint32_t pos = (uint32_t)(a.sup_offs[yb] + sex);
    double* sc = a.sup_cdf + (uint64_t)blockIdx.y * kSupportMax;
    uint64_t* si = a.sup_idx + (uint64_t)blockIdx.y * kSupportMax;
    for (uint32_t i = 0; i < per; ++i)
      if ((nz >> i) & 1u) {
        sc[pos] = v[i];
        si[pos] = e0 + tid * per + i;
        ++pos;
      }
  }
  __syncthreads();
  double* out = a.cdf ? a.cdf + (uint64_t)blockIdx.y * a.N : reinterpret_cast<double*>(st);
  if (E == kScanBlock) {
#pragma unroll
    for (uint32_t i = 0; i < kScanBlock / 256; ++i) out[e0 + tid + 256u * i] = sh[scan_pad(tid + 256u * i)];
  } else {
    for (uint32_t e = tid; e < E; e += blockDim.x) out[e0 + e] = sh[scan_pad(e)];
  }
}

// partial[t * nblk + b] = sum over block b of |psi|^2 (FP64).
template <typename V>
__global__ __launch_bounds__(256) void k_blocksum(ScanArgs<V> a) {
  block_prob_scan<V, false>(a);
}

// offs[t*nblk+b] = exclusive prefix of partial over blocks; total[t] = full sum.
// With support lists, the same for the blocks' nonzero counts (exact: integers
// below 2^53) and count[t] = the state's number of nonzero entries.
__device__ __forceinline__ double scan_blocks(const double* p, double* o, uint32_t nblk) {
  const uint32_t per = (nblk + 255) / 256;
  const uint32_t b0 = threadIdx.x * per;
  double s = 0.0;
  for (uint32_t i = 0; i < per; ++i)
    if (b0 + i < nblk) s += p[b0 + i];
  double ex, tot;
  block_excl_scan(s, &ex, &tot);
  double run = ex;
  for (uint32_t i = 0; i < per; ++i)
    if (b0 + i < nblk) {
      o[b0 + i] = run;
      run += p[b0 + i];
    }
  return run;
}

__global__ __launch_bounds__(256) void k_scan_partials(double* partial, double* offs, double* total, uint32_t nblk,
                                                       double* sup_part, double* sup_offs, uint32_t* sup_count,
                                                       const double* maxa, double* floor) {
  const uint64_t r0 = (uint64_t)blockIdx.x * nblk;
  const double run = scan_blocks(partial + r0, offs + r0, nblk);
  if (threadIdx.x == 255) total[blockIdx.x] = run;
  if (maxa) {
    // floor[b] = the largest CDF value of blocks 0 .. b-1: max over them of off + largest A
    __syncthreads();  // offs of every block written
    const uint32_t per = (nblk + 255) / 256;
    const uint32_t b0 = threadIdx.x * per;
    double m = 0.0;
    for (uint32_t i = 0; i < per; ++i)
      if (b0 + i < nblk) m = fmax(m, offs[r0 + b0 + i] + maxa[r0 + b0 + i]);
    double all;
    double run_max = block_excl_max(m, 0.0, &all);
    for (uint32_t i = 0; i < per; ++i)
      if (b0 + i < nblk) {
        floor[r0 + b0 + i] = run_max;
        run_max = fmax(run_max, offs[r0 + b0 + i] + maxa[r0 + b0 + i]);
      }
  }
  if (sup_part) {
    const double c = scan_blocks(sup_part + r0, sup_offs + r0, nblk);
    if (threadIdx.x == 255) sup_count[blockIdx.x] = c > (double)kSupportMax ? 0xffffffffu : (uint32_t)c;
  }
}

// Inclusive FP64 prefix sum of |psi|^2, written in place over each complex64
// slot (or to `cdf` for complex128).
template <typename V>
__global__ __launch_bounds__(256) void k_cdf(ScanArgs<V> a) {
  block_prob_scan<V, true>(a);
}

// ------------------------------------------------------------ adjoint sweep

// One unitary op of a tile pass on an LDS tile (all threads; caller syncs).
template <typename V>
__device__ __forceinline__ void tile_apply(V* tile, const DOp& op, const V* m, uint64_t base, uint32_t nt,
                                           uint32_t tid, uint32_t bd) {
  if (op.type == DOP_M1) {
    const V m00 = m[0], m01 = m[1], m10 = m[2], m11 = m[3];
    const uint32_t bit = 1u << op.a, lo = bit - 1;
    for (uint32_t pr = tid; pr < nt / 2; pr += bd) {
      const uint32_t i0 = ((pr & ~lo) << 1) | (pr & lo), i1 = i0 | bit;
      const V x0 = tile[i0], x1 = tile[i1];
      tile[i0] = cfma2(m00, x0, m01, x1);
      tile[i1] = cfma2(m10, x0, m11, x1);
    }
  } else if (op.type == DOP_M2) {
    const uint32_t A = 1u << op.a, B = 1u << op.b;
    const uint32_t l1 = min(A, B) - 1, l2 = max(A, B) - 1;
    for (uint32_t qd = tid; qd < nt / 4; qd += bd) {
      uint32_t i = ((qd & ~l1) << 1) | (qd & l1);
      i = ((i & ~l2) << 1) | (i & l2);
      const V x0 = tile[i], x1 = tile[i | A], x2 = tile[i | B], x3 = tile[i | A | B];
      tile[i] = cdot4(m, x0, x1, x2, x3);
      tile[i | A] = cdot4(m + 4, x0, x1, x2, x3);
      tile[i | B] = cdot4(m + 8, x0, x1, x2, x3);
      tile[i | A | B] = cdot4(m + 12, x0, x1, x2, x3);
    }
  } else if (op.type == DOP_D1 || op.type == DOP_D2) {
    const bool two = op.type == DOP_D2;
    const uint32_t dd = two ? 5 : 3;
    const uint32_t fa = op.a == 255 ? (uint32_t)((base >> op.ga) & 1) : 0;
    const uint32_t fb = (two && op.b == 255) ? (uint32_t)((base >> op.gb) & 1) : 0;
    for (uint32_t L = tid; L < nt; L += bd) {
      const uint32_t ba = op.a == 255 ? fa : (L >> op.a) & 1u;
      const uint32_t bb = two ? (op.b == 255 ? fb : (L >> op.b) & 1u) : 0;
      tile[L] = cmul(m[(ba + 2 * bb) * dd], tile[L]);
    }
  } else if (op.type == DOP_DSIGN) {
    const uint32_t fa = op.a == 255 ? (uint32_t)((base >> op.ga) & 1) : 0;
    const uint32_t fb = op.b == 255 ? (uint32_t)((base >> op.gb) & 1) : 0;
    for (uint32_t L = tid; L < nt; L += bd) {
      const uint32_t ba = op.a == 255 ? fa : (L >> op.a) & 1u;
      const uint32_t bb = op.b == 254 ? 0u : (op.b == 255 ? fb : (L >> op.b) & 1u);
      if ((op.slot[0] >> (ba + 2 * bb)) & 1u) {
        V v = tile[L];
        v.x = -v.x;
        v.y = -v.y;
        tile[L] = v;
      }
    }
  }
}

template <typename V>
__device__ __forceinline__ double im_conj_mul(V a, V b) {  // Im(conj(a) b)
  return (double)a.x * (double)b.y - (double)a.y * (double)b.x;
}
template <typename V>
__device__ __forceinline__ double re_conj_mul(V a, V b) {  // Re(conj(a) b)
  return (double)a.x * (double)b.x + (double)a.y * (double)b.y;
}

template <typename V>
__global__ __launch_bounds__(256) void k_adjoint(AdjArgs<V> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const PassArgs<V>& pa = a.p;
  const DPass& P = pa.passes[pa.pass];
  const uint32_t k = P.k, nt = 1u << k;
  V* tp = reinterpret_cast<V*>(smem);
  V* tl = tp + nt;
  uint32_t* slot_off = reinterpret_cast<uint32_t*>(tl + nt);
  __shared__ uint8_t tq[16];
  const uint32_t tid = threadIdx.x, bd = blockDim.x;
  const uint32_t t = pa.t0 + blockIdx.y;
  const uint64_t tile_id = blockIdx.x;
  if (tid < 16) tq[tid] = P.tq[tid];
  uint64_t base = 0;
  for (uint32_t i = 0; i < pa.n - k; ++i)
    if ((tile_id >> i) & 1) base |= 1ull << P.oq[i];
  V* sp = pa.states + (uint64_t)blockIdx.y * pa.N;
  V* sl = a.lam + (uint64_t)blockIdx.y * pa.N;
  for (uint32_t s = tid; s < P.n_slots; s += bd) slot_off[s] = pa.slot_default[P.slot_begin + s];
  __syncthreads();
  {
    const uint32_t ob = pa.ov_off[(uint64_t)t * pa.n_passes + pa.pass];
    const uint32_t oe = pa.ov_off[(uint64_t)t * pa.n_passes + pa.pass + 1];
    for (uint32_t i = ob + tid; i < oe; i += bd) slot_off[pa.ov[i].slot] = pa.ov[i].off;
  }
  for (uint32_t L = tid; L < nt; L += bd) {
    const uint64_t off = swizzle(base + tile_offset(L, tq, k), pa.swz);
    tp[L] = sp[off];
    tl[L] = sl[off];
  }
  __syncthreads();
  const DOp* ops = pa.ops + P.op_begin;
  // register-phase ops of a phased program act on the LDS tiles directly:
  // PHASE only renames the 4 register bits, M1G is up to 4 2x2 matrices on them,
  // signs are applied as they come (SFLIP has nothing left to do)
  uint32_t R[4] = {k - 4, k - 3, k - 2, k - 1};
  for (uint32_t o = 0; o < P.n_ops; ++o) {
    const DOp op = ops[o];
    if (op.type == DOP_PHASE) {
      R[0] = op.a;
      R[1] = op.b;
      R[2] = op.ga;
      R[3] = op.gb;
      continue;
    }
    if (op.type == DOP_SFLIP) continue;
    if (op.type == DOP_M1G) {
      for (uint32_t j = 0; j < 4; ++j) {
        if (!((op.mask >> j) & 1u)) continue;
        DOp m1{};
        m1.type = DOP_M1;
        m1.a = (uint8_t)R[j];
        const V* m = pa.pool + slot_off[op.slot[j]];
        tile_apply(tp, m1, m, base, nt, tid, bd);
        tile_apply(tl, m1, m, base, nt, tid, bd);
        __syncthreads();
      }
      continue;
    }
    if (op.type == DOP_DOT) {
      // Im<lambda|P_q|psi> restricted to this tile (pairs along local bit a)
      const uint32_t bit = 1u << op.a, lo = bit - 1;
      double acc = 0.0;
      for (uint32_t pr = tid; pr < nt / 2; pr += bd) {
        const uint32_t i0 = ((pr & ~lo) << 1) | (pr & lo), i1 = i0 | bit;
        const V l0 = tl[i0], l1 = tl[i1], p0 = tp[i0], p1 = tp[i1];
        if (op.b == 3)        // Z
          acc += im_conj_mul(l0, p0) - im_conj_mul(l1, p1);
        else if (op.b == 1)   // X
          acc += im_conj_mul(l0, p1) + im_conj_mul(l1, p0);
        else                  // Y: (Y psi)_0 = -i psi_1, (Y psi)_1 = i psi_0
          acc += re_conj_mul(l1, p0) - re_conj_mul(l0, p1);
      }
      double ex, tot;
      block_excl_scan(acc, &ex, &tot);
      const uint32_t d = (uint32_t)op.slot[0] | ((uint32_t)op.slot[1] << 16);
      if (tid == 0) a.partial[((uint64_t)t * gridDim.x + tile_id) * a.n_dot + d] = tot;
    } else {
      // DSIGN carries its sign mask in slot[0] and reads no matrix
      const V* m = op.type == DOP_DSIGN ? pa.pool : pa.pool + slot_off[op.slot[0]];
      tile_apply(tp, op, m, base, nt, tid, bd);
      tile_apply(tl, op, m, base, nt, tid, bd);
    }
    __syncthreads();
  }
  for (uint32_t L = tid; L < nt; L += bd) {
    const uint64_t off = base + tile_offset(L, tq, k);
    sp[off] = tp[L];
    sl[off] = tl[L];
  }
}

// lambda <- (s K_k)^dagger lambda on qubit q (FP64 matrix): the adjoint of the
// operator a state-dependent channel applied in the forward sweep, held fixed.
template <typename V>
__global__ __launch_bounds__(256) void k_gch_lam_adjoint(GchAdjArgs<V> a) {
  const uint64_t ri = (uint64_t)(a.t0 + blockIdx.y) * a.n_measure + a.rec;
  const uint32_t kk = a.mr_bits[ri];
  const double sc = a.mr_norm[ri];
  const double* K = a.chan + 1 + 2 * (uint32_t)a.chan[0] + 8 * kk;  // K_k row-major, re/im
  // (K^dagger)_{ij} = conj(K_{ji})
  const double h00r = sc * K[0], h00i = -sc * K[1];
  const double h01r = sc * K[4], h01i = -sc * K[5];
  const double h10r = sc * K[2], h10i = -sc * K[3];
  const double h11r = sc * K[6], h11i = -sc * K[7];
  V* l = a.lam + (uint64_t)blockIdx.y * a.N;
  const uint64_t bit = 1ull << a.q, lo = bit - 1;
  for (uint64_t pr = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; pr < a.N / 2;
       pr += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t c0 = ((pr & ~lo) << 1) | (pr & lo);
    const uint64_t i0 = swizzle(c0, a.swz), i1 = swizzle(c0 | bit, a.swz);
    const V x0 = l[i0], x1 = l[i1];
    const double ar = x0.x, ai = x0.y, br = x1.x, bi = x1.y;
    V y0, y1;
    y0.x = (typename Real<V>::T)(h00r * ar - h00i * ai + h01r * br - h01i * bi);
    y0.y = (typename Real<V>::T)(h00r * ai + h00i * ar + h01r * bi + h01i * br);
    y1.x = (typename Real<V>::T)(h10r * ar - h10i * ai + h11r * br - h11i * bi);
    y1.y = (typename Real<V>::T)(h10r * ai + h10i * ar + h11r * bi + h11i * br);
    l[i0] = y0;
    l[i1] = y1;
  }
}

// lambda = O psi for a diagonal O = sum_t coef_t Z-string(zmask_t)
template <typename V>
__global__ __launch_bounds__(256) void k_obs_apply(ObsArgs<V> a) {
  const V* p = a.psi + (uint64_t)blockIdx.y * a.N;
  V* l = a.lam + (uint64_t)blockIdx.y * a.N;
  for (uint64_t pos = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; pos < a.N;
       pos += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x = swizzle(pos, a.swz);  // the amplitude stored at pos (an involution)
    double o = 0.0;
    for (uint32_t j = 0; j < a.n_terms; ++j) o += (__popcll(x & a.zmask[j]) & 1) ? -a.coef[j] : a.coef[j];
    V v = p[pos];
    v.x = (typename Real<V>::T)((double)v.x * o);
    v.y = (typename Real<V>::T)((double)v.y * o);
    l[pos] = v;
  }
}

__global__ void k_grad_dot(const double* partial, const double* w, uint32_t n_traj, uint32_t n_tiles, uint32_t n_dot,
                           double* gdot) {
  const uint32_t d = blockIdx.x;
  double s = 0.0;  // fixed order: thread-strided over trajectories, then the block tree
  for (uint32_t t = threadIdx.x; t < n_traj; t += blockDim.x) {
    double st = 0.0;
    for (uint32_t tile = 0; tile < n_tiles; ++tile) st += partial[((uint64_t)t * n_tiles + tile) * n_dot + d];
    s += w[t] * st;
  }
  double ex, tot;
  block_excl_scan(s, &ex, &tot);
  if (threadIdx.x == 0) gdot[d] = tot;
}

__global__ void k_grad_gather(const double* gdot, const uint32_t* dot_param, uint32_t n_dot, uint32_t n_params,
                              double* grad, const double* ev, const double* w, uint32_t n_traj, double* E) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n_params) {
    double g = 0.0;
    for (uint32_t d = 0; d < n_dot; ++d)
      if (dot_param[d] == p) g += gdot[d];
    grad[p] = g;
  }
  if (p == 0) {
    double e = 0.0;
    for (uint32_t t = 0; t < n_traj; ++t) e += w[t] * ev[t];
    *E = e;
  }
}

// ------------------------------------------------------------ measure-reset

template <typename V>
__global__ __launch_bounds__(256) void k_marginal(MarginalArgs<V> a) {
  const V* st = a.states + (uint64_t)(a.rows ? a.rows[blockIdx.y].x : blockIdx.y) * a.N;
  const uint64_t e0 = (uint64_t)blockIdx.x * a.per_block;
  // sums in registers: every index into s is a compile-time constant
  double s[kMaxGroup + 1];
#pragma unroll
  for (int j = 0; j <= kMaxGroup; ++j) s[j] = 0.0;
  auto add = [&](uint64_t x, double w) {
    s[0] += w;
#pragma unroll
    for (int j = 0; j < kMaxGroup; ++j)
      if (j < (int)a.nq && ((x >> a.q[j]) & 1)) s[j + 1] += w;
  };
  if (a.per_block == kScanBlock) {
    // full block: a thread's 16 loads in flight before the first use.  Its
    // amplitudes x = e0 + tid + 256 i differ only in index bits 8..11 (the bits
    // of i), so the thread forms its total and the four sums over i with bit b
    // set, and a measured qubit takes one of them (bits 8..11) or the total or
    // nothing (every other bit is fixed for the thread): the same sums, added
    // in the same order, as accumulating amplitude by amplitude.
    constexpr uint32_t kPer = kScanBlock / 256;
    const uint32_t sx = swizzle_block(blockIdx.x, a.swz);
    double w[kPer];
#pragma unroll
    for (uint32_t i = 0; i < kPer; ++i) w[i] = norm2(st[e0 + ((threadIdx.x + 256u * i) ^ sx)]);
    double tot = 0.0, sb[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (uint32_t i = 0; i < kPer; ++i) {
      tot += w[i];
#pragma unroll
      for (uint32_t b = 0; b < 4; ++b)
        if ((i >> b) & 1u) sb[b] += w[i];
    }
    const uint64_t xt = e0 + threadIdx.x;
    s[0] = tot;
#pragma unroll
    for (int j = 0; j < kMaxGroup; ++j)
      if (j < (int)a.nq) {
        const uint32_t q = a.q[j];
        const double in_thread = q == 8u ? sb[0] : q == 9u ? sb[1] : q == 10u ? sb[2] : sb[3];  // no indexed registers
        s[j + 1] = (q >= 8u && q < 12u) ? in_thread : (((xt >> q) & 1ull) ? tot : 0.0);
      }
  } else {
    for (uint32_t i = threadIdx.x; i < a.per_block; i += blockDim.x) add(e0 + i, norm2(st[e0 + i]));
  }
  // block totals of the nq + 1 sums: a wavefront butterfly per sum, then one
  // LDS exchange and one barrier for all of them
  __shared__ double wtot[4][kMaxGroup + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j <= kMaxGroup; ++j) {
    if (j <= (int)a.nq) {  // uniform over the block
      double v = s[j];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) wtot[wv][j] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x <= a.nq) {
    const uint32_t j = threadIdx.x;
    a.partial[((uint64_t)blockIdx.y * a.nblk + blockIdx.x) * (kMaxGroup + 1) + j] =
        ((wtot[0][j] + wtot[1][j]) + wtot[2][j]) + wtot[3][j];
  }
}

__global__ void k_mr_decide(MrDecideArgs a) {
  const uint32_t tb = blockIdx.x;  // batch-local trajectory, or entry tb of a.rows
  const uint32_t j = threadIdx.x;
  if (j >= a.nq) return;
  double tot = 0.0, one = 0.0;
  for (uint32_t b = 0; b < a.nblk; ++b) {
    const double* p = a.partial + ((uint64_t)tb * a.nblk + b) * (kMaxGroup + 1);
    tot += p[0];
    one += p[j + 1];
  }
  const double p1 = one / tot;
  // an empty or non-finite state leaves no valid decision: report it
  if (!(tot > 0.0) || !isfinite(p1)) atomicOr(a.status, 2u);
  const bool norm_here = j == 0 && a.carries_norm != 0;
  const uint32_t r = a.idx[j];
  const uint32_t co = a.rec_chan ? a.rec_chan[r] : 0xffffffffu;
  if (co != 0xffffffffu) {
    // state-dependent channel (never with a.rows: such plans share no prefix):
    // p_k = d0[k] P(q=0) + d1[k] P(q=1); the uniform is word rec_gidx[r] of the
    // stream [seed, key1(4, cfg, alpha)]
    const double* cp = a.chan_param + co;
    const uint32_t K = (uint32_t)cp[0];
    const uint64_t alpha = a.alpha0 + a.t0 + tb;
    const uint64_t g = a.rec_gidx[r];
    const U64x4 w = philox4x64_10(g / 4 + 1, 0, 0, 0, a.seed, stream_key1(4, a.cfg, alpha));
    const double u = word_to_uniform(w.v[g % 4]);
    // smallest k with u < p_0 + ... + p_k; past the end (rounding), the last k with p_k > 0
    uint32_t k = 0, k_last = 0;
    double c = 0.0, pk = 0.0, p_last = 0.0;
    bool found = false;
    for (uint32_t kk = 0; kk < K; ++kk) {
      const double p = cp[1 + kk] * (1.0 - p1) + cp[1 + K + kk] * p1;
      c += p;
      if (p > 0.0) {
        k_last = kk;
        p_last = p;
      }
      if (!found && u < c && p > 0.0) {
        k = kk;
        pk = p;
        found = true;
      }
    }
    if (!found) {
      k = k_last;
      pk = p_last;
    }
    const uint64_t ri = (uint64_t)(a.t0 + tb) * a.n_measure + r;
    a.mr_bits[ri] = (uint8_t)k;
    a.mr_norm[ri] = norm_here ? 1.0 / sqrt(pk * tot) : 1.0 / sqrt(pk);
    return;
  }
  const uint32_t bit = p1 > 0.5 ? 1u : 0u;
  const double pb = bit ? p1 : 1.0 - p1;
  if (fmin(p1, 1.0 - p1) > a.tol) atomicOr(a.status, 1u);
  // Every measure-reset of the step scales the whole state once; the step's
  // first one also carries the 1/||psi|| renormalisation.
  const double sc = norm_here ? 1.0 / sqrt(pb * tot) : 1.0 / sqrt(pb);
  const uint32_t row = a.rows == nullptr                ? a.t0 + tb
                       : a.rows[tb].y >= a.carrier0 ? a.carrier_t
                                                    : a.t0 + a.rows[tb].y;
  const uint64_t ri = (uint64_t)row * a.n_measure + a.idx[j];
  a.mr_bits[ri] = (uint8_t)bit;
  a.mr_norm[ri] = sc;
}

// Trajectories still on the error-free prefix at a decision step hold the
// prefix state, so they take its decisions: copy the group's entries of the
// prefix state's record row to theirs (one thread per batch trajectory).
__global__ void k_mr_follow(MrDecideArgs a) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.bb || a.eff[a.t0 + b] <= a.step) return;
  const uint64_t src = (uint64_t)a.carrier_t * a.n_measure, dst = (uint64_t)(a.t0 + b) * a.n_measure;
  for (uint32_t j = 0; j < a.nq; ++j) {
    a.mr_bits[dst + a.idx[j]] = a.mr_bits[src + a.idx[j]];
    a.mr_norm[dst + a.idx[j]] = a.mr_norm[src + a.idx[j]];
  }
}

// ------------------------------------------------------------------ sampler

// One register stage of the bitonic network on a thread's 16 elements
// 16c .. 16c + 15: pairs (r, r + stride) for (r & stride) == 0, ascending where
// ((16c + r) & size) == 0.  Called with constant stride (unrolled) so x stays
// in registers.
__device__ __forceinline__ void sort_stage_regs(double (&x)[16], uint32_t size, uint32_t stride, uint32_t c) {
#pragma unroll
  for (uint32_t r = 0; r < 16; ++r) {
    if (r & stride) continue;
    const uint32_t h = r | stride;
    const bool up = (((16u * c + r) & size) == 0);
    const double xa = x[r], xb = x[h];
    if ((xa > xb) == up) {
      x[r] = xb;
      x[h] = xa;
    }
  }
}

// A chunk of a trajectory whose state has a short support list (at most
// kSupportMax elements that an upper-bound search can return): the same
// uniforms, each searched in the list held in LDS, counted per list element,
// and written out as the counts' runs in ascending order -- the sorted chunk
// of the full path, since the search result is monotone in u.  `sh` is the
// block's 32 KiB of LDS.
template <typename BitT>
__device__ void sample_support(const SampleArgs<BitT>& a, double* sh, uint32_t t, uint64_t j0, uint32_t cnt,
                               uint64_t alpha, uint64_t k1, uint64_t out0) {
  const uint32_t tb = t - a.b0;
  const uint32_t K = a.sup_count[tb];
  double* scdf = sh;                                                      // K CDF values
  uint64_t* sidx = reinterpret_cast<uint64_t*>(sh + kSupportMax);         // K basis indices
  uint32_t* hist = reinterpret_cast<uint32_t*>(sh + 2 * kSupportMax);     // K + 1 counts
  uint32_t* hoff = hist + kSupportMax + 4;                                // K + 2 run starts
  const double* gsc = a.sup_cdf + (uint64_t)tb * kSupportMax;
  const uint64_t* gsi = a.sup_idx + (uint64_t)tb * kSupportMax;
  for (uint32_t i = threadIdx.x; i < K; i += blockDim.x) {
    scdf[i] = gsc[i];
    sidx[i] = gsi[i];
  }
  for (uint32_t i = threadIdx.x; i <= K; i += blockDim.x) hist[i] = 0u;
  __syncthreads();
  const double total = a.total[tb];
  for (uint32_t i = threadIdx.x * 4; i < cnt; i += blockDim.x * 4) {
    double uu[4];
    if (a.uniforms) {
      for (int w = 0; w < 4; ++w) uu[w] = (i + w < cnt) ? a.uniforms[out0 + i + w] : 0.0;
    } else {
      const U64x4 r = philox4x64_10((j0 + i) / 4 + 1, 0, 0, 0, a.seed, k1);
      for (int w = 0; w < 4; ++w) uu[w] = word_to_uniform(r.v[w]);
    }
    for (int w = 0; w < 4; ++w) {
      if (i + w >= cnt) break;
      const double v = uu[w] * total;
      uint32_t lo = 0, h = K;
      while (lo < h) {
        const uint32_t mid = (lo + h) >> 1;
        if (scdf[mid] > v)
          h = mid;
        else
          lo = mid + 1;
      }
      atomicAdd(hist + lo, 1u);   // lo == K: no element exceeds v (the full search clamps to N - 1)
    }
  }
  __syncthreads();
  // run starts: exclusive prefix of the K + 1 counts
  const uint32_t nb = K + 1, per = (nb + blockDim.x - 1) / blockDim.x, c0 = threadIdx.x * per;
  double sum = 0.0;
  for (uint32_t q = 0; q < per; ++q)
    if (c0 + q < nb) sum += (double)hist[c0 + q];
  double ex, tot;
  block_excl_scan(sum, &ex, &tot);
  uint32_t run = (uint32_t)ex;
  for (uint32_t q = 0; q < per; ++q)
    if (c0 + q < nb) {
      hoff[c0 + q] = run;
      run += hist[c0 + q];
    }
  if (threadIdx.x == 0) hoff[nb] = cnt;
  __syncthreads();
  const uint64_t N = a.N;
  // each output position j takes the last run starting at or before j (empty
  // runs start where the next one does): a bisection for the thread's first
  // position, then a forward walk, since its positions only increase
  // (hoff[nb] = cnt > j ends every walk)
  uint32_t lo = 0;
  if (threadIdx.x < cnt) {
    uint32_t h = nb;
    while (h - lo > 1) {
      const uint32_t mid = (lo + h) >> 1;
      if (hoff[mid] <= threadIdx.x)
        lo = mid;
      else
        h = mid;
    }
  }
  for (uint32_t j = threadIdx.x; j < cnt; j += blockDim.x) {
    while (hoff[lo + 1] <= j) ++lo;
    const uint64_t l = lo < K ? sidx[lo] : N - 1;
    a.bits[out0 + j] = (BitT)l;
    a.traj[out0 + j] = (uint32_t)alpha;
  }
}

template <typename BitT>
__global__ __launch_bounds__(256) void k_sample(SampleArgs<BitT> a) {
  __shared__ double u[4096];
  const uint64_t item = a.item0 + blockIdx.x;
  // trajectory of this item: chunk_off[t] <= item < chunk_off[t+1], t in [b0, b1)
  uint32_t lo = a.b0, hi = a.b1;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (a.chunk_off[mid] <= item)
      lo = mid;
    else
      hi = mid;
  }
  const uint32_t t = lo;
  const uint64_t c = item - a.chunk_off[t];
  const uint64_t m = a.shot_off[t + 1] - a.shot_off[t];
  const uint32_t C = a.chunk;
  const uint64_t j0 = c * C;
  const uint32_t cnt = (uint32_t)min((uint64_t)C, m - j0);
  const uint64_t alpha = a.alpha0 + t;
  const uint64_t k1 = stream_key1(2, a.cfg, alpha);
  const uint64_t out0 = a.shot_off[t] + j0;
  if (a.sup_count && a.sup_count[t - a.b0] <= kSupportMax) {
    sample_support(a, u, t, j0, cnt, alpha, k1, out0);
    return;
  }
  // Element i of the chunk lives at LDS index (i & 15) * R + (i >> 4), R = C / 16
  // columns: thread col < R holds elements 16 col .. 16 col + 15 of a row-major 16 x R
  // view, so register loads, column-pair LDS stages and the uniforms' stores
  // are bank-conflict free.
  const uint32_t R = C >> 4;
  // uniforms: shot j uses word j of the trajectory's sampler stream
  for (uint32_t i = threadIdx.x * 4; i < C; i += blockDim.x * 4) {
    if (a.uniforms) {
      for (int w = 0; w < 4; ++w) u[((i + w) & 15u) * R + ((i + w) >> 4)] = (i + w < cnt) ? a.uniforms[out0 + i + w] : 2.0;
    } else {
      const uint64_t j = j0 + i;  // multiple of 4 because C and i are
      U64x4 r = philox4x64_10(j / 4 + 1, 0, 0, 0, a.seed, k1);
      for (int w = 0; w < 4; ++w)
        u[((i + w) & 15u) * R + ((i + w) >> 4)] = (i + w < cnt) ? word_to_uniform(r.v[w]) : 2.0;
    }
  }
  __syncthreads();
  // Bitonic sort of the C values (padding 2.0 sorts last): every stage compares
  // elements i and i + stride for (i & stride) == 0, ascending where
  // (i & size) == 0.  Strides below 16 pair elements of one thread and run in
  // registers; larger strides pair columns of one row in LDS.
  const uint32_t col = threadIdx.x;
  const bool holder = col < R;
  double x[16];
  if (holder) {
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = u[r * R + col];
#pragma unroll
    for (uint32_t size = 2; size <= 16; size <<= 1)
#pragma unroll
      for (uint32_t stride = size >> 1; stride > 0; stride >>= 1)
        sort_stage_regs(x, size, stride, col);
#pragma unroll
    for (int r = 0; r < 16; ++r) u[r * R + col] = x[r];
  }
  __syncthreads();
  for (uint32_t size = 32; size <= C; size <<= 1) {
    for (uint32_t stride = size >> 1; stride >= 16; stride >>= 1) {
      const uint32_t sc = stride >> 4, half = R >> 1;
      for (uint32_t q = threadIdx.x; q < C / 2; q += blockDim.x) {
        const uint32_t row = q / half, pc = q - row * half;
        const uint32_t lo_c = 2 * pc - (pc & (sc - 1)), hi_c = lo_c + sc;
        const bool up = (((lo_c << 4) & size) == 0);
        const double xa = u[row * R + lo_c], xb = u[row * R + hi_c];
        if ((xa > xb) == up) {
          u[row * R + lo_c] = xb;
          u[row * R + hi_c] = xa;
        }
      }
      __syncthreads();
    }
    if (holder) {
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = u[r * R + col];
#pragma unroll
      for (uint32_t stride = 8; stride > 0; stride >>= 1) sort_stage_regs(x, size, stride, col);
#pragma unroll
      for (int r = 0; r < 16; ++r) u[r * R + col] = x[r];
    }
    __syncthreads();
  }
  // Each thread takes g = ceil(cnt / blockDim) consecutive elements of the
  // sorted chunk: the first is found by bisection, each next one from the
  // previous result on (exponential probe, then bisection), since its answer
  // can only be at or after it.  The index found is the first with
  // cdf > u * total, as a bisection from 0 finds.  A thread reads and then
  // overwrites only its own elements' LDS slots with the results, which go out
  // after the barrier in coalesced stores.
  const double* cdf = a.cdf_base + (uint64_t)(t - a.b0) * a.cdf_stride;
  const double total = a.total[t - a.b0];
  const uint64_t N = a.N;
  {
    const uint32_t g = (cnt + blockDim.x - 1) / blockDim.x;
    const uint32_t e0 = threadIdx.x * g, e1 = min(cnt, e0 + g);
    uint64_t p = 0;
    for (uint32_t e = e0; e < e1; ++e) {
      const uint32_t li = (e & 15u) * R + (e >> 4);
      const double v = u[li] * total;
      uint64_t lo = e == e0 ? 0 : p, h = N;
      if (e != e0) {
        uint64_t probe = lo, step = 1;
        while (probe < N && !(cdf[probe] > v)) {
          lo = probe + 1;
          probe = lo + step;
          step <<= 1;
        }
        h = probe < N ? probe : N;
      }
      while (lo < h) {
        const uint64_t mid = (lo + h) >> 1;
        if (cdf[mid] > v)
          h = mid;
        else
          lo = mid + 1;
      }
      p = lo;
      u[li] = __longlong_as_double((long long)p);
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
    uint64_t l = (uint64_t)__double_as_longlong(u[(i & 15u) * R + (i >> 4)]);
    if (l > N - 1) l = N - 1;
    a.bits[out0 + i] = (BitT)l;
    a.traj[out0 + i] = (uint32_t)alpha;
  }
}

// ------------------------------------------------------------ states / <O>

template <typename V>
__global__ __launch_bounds__(256) void k_copy_normalised(const V* states, V* out, const double* total, uint64_t N,
                                                         uint32_t swz) {
  const double s = 1.0 / sqrt(total[blockIdx.y]);
  const V* st = states + (uint64_t)blockIdx.y * N;
  V* o = out + (uint64_t)blockIdx.y * N;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x) {
    V v = st[swizzle(i, swz)];
    v.x = (typename Real<V>::T)((double)v.x * s);
    v.y = (typename Real<V>::T)((double)v.y * s);
    o[i] = v;
  }
}

template <typename V>
__global__ __launch_bounds__(256) void k_expval(ExpArgs<V> a) {
  const V* st = a.states + (uint64_t)blockIdx.y * a.N;
  const uint64_t e0 = (uint64_t)blockIdx.x * a.per_block;
  double s = 0.0;
  for (uint32_t i = threadIdx.x; i < a.per_block; i += blockDim.x) {
    const uint64_t x = e0 + i;
    double o = 0.0;
    for (uint32_t j = 0; j < a.n_terms; ++j)
      o += (__popcll(x & a.zmask[j]) & 1) ? -a.coef[j] : a.coef[j];
    s += norm2(st[swizzle(x, a.swz)]) * o;
  }
  double ex, tot;
  block_excl_scan(s, &ex, &tot);
  if (threadIdx.x == 0) a.partial[(uint64_t)blockIdx.y * a.nblk + blockIdx.x] = tot;
}

__global__ void k_expval_finish(const double* partial, const double* total, double* out, uint32_t nblk, uint32_t t0) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (uint32_t b = 0; b < nblk; ++b) s += partial[(uint64_t)blockIdx.x * nblk + b];
  out[t0 + blockIdx.x] = s / total[blockIdx.x];
}

// E = sum_t w[t] ev[t], summed in trajectory order (the order the adjoint
// gradient's value uses).
__global__ void k_weighted_sum(const double* w, const double* ev, uint32_t n, double* E) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double e = 0.0;
  for (uint32_t t = 0; t < n; ++t) e += w[t] * ev[t];
  *E = e;
}

// ------------------------------------------- dense state-dependent channels

// Index with zeros inserted at the channel's qubit positions (ascending), the
// amplitudes of base j being base | a-th combination of those bits.
__device__ __forceinline__ uint64_t insert_zero(uint64_t j, uint32_t q) {
  return ((j >> q) << (q + 1)) | (j & ((1ull << q) - 1));
}
template <typename V>
__device__ __forceinline__ uint64_t dense_base(const DenseArgs<V>& a, uint64_t j) {
  if (a.nq == 1) return insert_zero(j, a.q[0]);
  const uint32_t lo = min(a.q[0], a.q[1]), hi = max(a.q[0], a.q[1]);
  return insert_zero(insert_zero(j, lo), hi);
}
template <typename V>
__device__ __forceinline__ uint64_t dense_index(const DenseArgs<V>& a, uint64_t base, uint32_t i) {
  uint64_t x = base;
  if (i & 1u) x |= 1ull << a.q[0];
  if (i & 2u) x |= 1ull << a.q[1];
  return x;
}

// Partial sums of rho[i][j] = sum psi_i conj(psi_j), i <= j, over one block of
// base indices: 16 slots (diagonal real parts, then re/im of the upper entries).
template <typename V>
__global__ __launch_bounds__(256) void k_rdm(DenseArgs<V> a) {
  const uint32_t d = 1u << a.nq;
  const V* st = a.states + (uint64_t)blockIdx.y * a.N;
  const uint64_t NB = a.N >> a.nq;
  double acc[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) acc[c] = 0.0;
  for (uint32_t it = 0; it < 16; ++it) {
    const uint64_t j = (uint64_t)blockIdx.x * 4096u + threadIdx.x + 256u * it;
    if (j >= NB) break;
    const uint64_t b = dense_base(a, j);
    double re[4], im[4];
    for (uint32_t i = 0; i < d; ++i) {
      const V v = st[swizzle(dense_index(a, b, i), a.swz)];
      re[i] = (double)v.x;
      im[i] = (double)v.y;
    }
    int c = 0;
    for (uint32_t i = 0; i < d; ++i) acc[c++] += re[i] * re[i] + im[i] * im[i];
    for (uint32_t i = 0; i < d; ++i)
      for (uint32_t k = i + 1; k < d; ++k) {
        acc[c++] += re[i] * re[k] + im[i] * im[k];   // Re psi_i conj(psi_k)
        acc[c++] += im[i] * re[k] - re[i] * im[k];   // Im psi_i conj(psi_k)
      }
  }
  __shared__ double wsum[4][16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    double v = acc[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) wsum[w][c] = v;
  }
  __syncthreads();
  if (threadIdx.x < 16) {
    const double v = ((wsum[0][threadIdx.x] + wsum[1][threadIdx.x]) + wsum[2][threadIdx.x]) + wsum[3][threadIdx.x];
    a.partial[((uint64_t)blockIdx.y * a.nblk + blockIdx.x) * 16 + threadIdx.x] = v;
  }
}

template <typename V>
__global__ void k_dense_decide(DenseArgs<V> a) {
  const uint32_t tb = blockIdx.x;
  __shared__ double comp[16];
  if (threadIdx.x < 16) {
    double v = 0.0;
    for (uint32_t b = 0; b < a.nblk; ++b) v += a.partial[((uint64_t)tb * a.nblk + b) * 16 + threadIdx.x];
    comp[threadIdx.x] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const uint32_t d = 1u << a.nq;
  // rho as d x d complex (upper entries from the slots, lower by conjugation)
  double rr[16], ri[16];
  int c = 0;
  for (uint32_t i = 0; i < d; ++i) {
    rr[i * d + i] = comp[c++];
    ri[i * d + i] = 0.0;
  }
  for (uint32_t i = 0; i < d; ++i)
    for (uint32_t k = i + 1; k < d; ++k) {
      rr[i * d + k] = comp[c];
      rr[k * d + i] = comp[c++];
      ri[i * d + k] = comp[c];
      ri[k * d + i] = -comp[c++];
    }
  double tot = 0.0;
  for (uint32_t i = 0; i < d; ++i) tot += rr[i * d + i];
  const uint32_t K = (uint32_t)a.chan[0];
  const double* M = a.chan + 2;
  const uint64_t alpha = a.alpha0 + a.t0 + tb;
  const U64x4 w = philox4x64_10(a.gidx / 4 + 1, 0, 0, 0, a.seed, stream_key1(4, a.cfg, alpha));
  const double u = word_to_uniform(w.v[a.gidx % 4]);
  uint32_t kk = 0, k_last = 0;
  double cum = 0.0, pk = 0.0, p_last = 0.0;
  bool found = false;
  for (uint32_t k = 0; k < K; ++k) {
    // Re Tr(M_k rho) = sum_ij Re(M_ij rho_ji)
    const double* m = M + (uint64_t)k * 2 * d * d;
    double t = 0.0;
    for (uint32_t i = 0; i < d; ++i)
      for (uint32_t j = 0; j < d; ++j)
        t += m[2 * (i * d + j)] * rr[j * d + i] - m[2 * (i * d + j) + 1] * ri[j * d + i];
    const double p = t / tot;
    cum += p;
    if (p > 0.0) {
      k_last = k;
      p_last = p;
    }
    if (!found && u < cum && p > 0.0) {
      kk = k;
      pk = p;
      found = true;
    }
  }
  if (!found) {
    kk = k_last;
    pk = p_last;
  }
  if (!(tot > 0.0) || !isfinite(tot) || !(pk > 0.0)) atomicOr(a.status, 2u);
  const uint64_t ri2 = (uint64_t)(a.t0 + tb) * a.n_measure + a.rec;
  a.mr_bits[ri2] = (uint8_t)kk;
  a.mr_norm[ri2] = 1.0 / sqrt(pk * tot);
}

// psi <- factor K_k psi (forward) or lambda <- factor K_k^dagger lambda (reverse)
template <typename V, bool kAdjoint>
__global__ __launch_bounds__(256) void k_dense_apply(DenseArgs<V> a) {
  const uint32_t d = 1u << a.nq;
  const uint64_t ri = (uint64_t)(a.t0 + blockIdx.y) * a.n_measure + a.rec;
  const uint32_t kk = a.mr_bits[ri];
  const double sc = a.mr_norm[ri];
  const uint32_t K = (uint32_t)a.chan[0];
  const double* G = a.chan + 2 + 2ull * d * d * (K + kk);
  double gr[16], gi[16];
  for (uint32_t i = 0; i < d; ++i)
    for (uint32_t j = 0; j < d; ++j) {
      // forward: (s K)_ij; reverse: (s K)^dagger_ij = s conj(K_ji)
      const uint32_t e = kAdjoint ? j * d + i : i * d + j;
      gr[i * d + j] = sc * G[2 * e];
      gi[i * d + j] = kAdjoint ? -sc * G[2 * e + 1] : sc * G[2 * e + 1];
    }
  V* st = (kAdjoint ? a.lam : a.states) + (uint64_t)blockIdx.y * a.N;
  const uint64_t NB = a.N >> a.nq;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < NB; j += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t b = dense_base(a, j);
    uint64_t pos[4];
    double xr[4], xi[4];
    for (uint32_t i = 0; i < d; ++i) {
      pos[i] = swizzle(dense_index(a, b, i), a.swz);
      const V v = st[pos[i]];
      xr[i] = v.x;
      xi[i] = v.y;
    }
    for (uint32_t i = 0; i < d; ++i) {
      double yr = 0.0, yi = 0.0;
      for (uint32_t k = 0; k < d; ++k) {
        yr += gr[i * d + k] * xr[k] - gi[i * d + k] * xi[k];
        yi += gr[i * d + k] * xi[k] + gi[i * d + k] * xr[k];
      }
      V y;
      y.x = (typename Real<V>::T)yr;
      y.y = (typename Real<V>::T)yi;
      st[pos[i]] = y;
    }
  }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// -------------------------------------------------------------- launchers

template <typename V>
hipError_t launch_pass(const PassArgs<V>& a, uint32_t k, uint32_t n_slots, uint32_t n_ops, uint32_t batch,
                       hipStream_t s) {
  dim3 grid(1u << (a.n - k), batch);
  if (k >= kMinRegTile && k <= 12) {
    const size_t lds = reg_lds_bytes<V>(k, n_slots, n_ops);
    if (lds > 65536) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_pass_reg<V>, grid, dim3(1u << (k - kRegBits)), lds, s, a);
  } else {
    const size_t lds = sizeof(V) * (size_t(1) << k) + 4 * (size_t)n_slots;
    if (lds > 65536) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_pass<V>, grid, dim3(256), lds, s, a);
  }
  return hipGetLastError();
}

template <typename V>
hipError_t launch_scan(const ScanArgs<V>& a, uint32_t batch, double* total, hipStream_t s) {
  dim3 grid(a.nblk, batch);
  hipLaunchKernelGGL(k_blocksum<V>, grid, dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_scan_partials, dim3(batch), dim3(256), 0, s, a.partial, a.offs, total, a.nblk, a.sup_part,
                     a.sup_offs, a.sup_count, a.maxa, a.floor);
  hipLaunchKernelGGL(k_cdf<V>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename V>
hipError_t launch_norm(const ScanArgs<V>& a, uint32_t batch, double* total, hipStream_t s) {
  dim3 grid(a.nblk, batch);
  ScanArgs<V> b = a;
  b.sup_part = nullptr;
  b.maxa = nullptr;
  hipLaunchKernelGGL(k_blocksum<V>, grid, dim3(256), 0, s, b);
  hipLaunchKernelGGL(k_scan_partials, dim3(batch), dim3(256), 0, s, b.partial, b.offs, total, b.nblk, nullptr,
                     nullptr, nullptr, nullptr, nullptr);
  return hipGetLastError();
}

template <typename V>
hipError_t launch_marginal(const MarginalArgs<V>& a, const MrDecideArgs& d, uint32_t batch, hipStream_t s) {
  hipLaunchKernelGGL(k_marginal<V>, dim3(a.nblk, batch), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_mr_decide, dim3(batch), dim3(64), 0, s, d);
  if (d.rows && d.eff && d.bb) hipLaunchKernelGGL(k_mr_follow, dim3((d.bb + 255) / 256), dim3(256), 0, s, d);
  return hipGetLastError();
}

template <typename BitT>
hipError_t launch_sample(const SampleArgs<BitT>& a, uint64_t items, hipStream_t s) {
  const uint64_t maxg = 0x7fffffffull;
  for (uint64_t done = 0; done < items; done += maxg) {
    SampleArgs<BitT> b = a;
    b.item0 = a.item0 + done;
    uint64_t g = items - done < maxg ? items - done : maxg;
    hipLaunchKernelGGL(k_sample<BitT>, dim3((uint32_t)g), dim3(256), 0, s, b);
  }
  return hipGetLastError();
}

template <typename V>
hipError_t launch_copy_normalised(const V* states, V* out, const double* total, uint64_t N, uint32_t batch,
                                  uint32_t swz, hipStream_t s) {
  uint32_t gx = (uint32_t)((N + 255) / 256 < 65536 ? (N + 255) / 256 : 65536);
  hipLaunchKernelGGL(k_copy_normalised<V>, dim3(gx, batch), dim3(256), 0, s, states, out, total, N, swz);
  return hipGetLastError();
}

template <typename V>
hipError_t launch_expval(const ExpArgs<V>& a, const double* total, double* out, uint32_t batch, uint32_t t0,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_expval<V>, dim3(a.nblk, batch), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_expval_finish, dim3(batch), dim3(64), 0, s, a.partial, total, out, a.nblk, t0);
  return hipGetLastError();
}

template <typename V>
hipError_t launch_adjoint_pass(const AdjArgs<V>& a, uint32_t k, uint32_t n_slots, uint32_t batch, hipStream_t s) {
  const size_t lds = 2 * sizeof(V) * (size_t(1) << k) + 4 * (size_t)n_slots;
  if (lds > 65536) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_adjoint<V>, dim3(1u << (a.p.n - k), batch), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <typename V>
hipError_t launch_obs_apply(const ObsArgs<V>& a, uint32_t batch, hipStream_t s) {
  uint32_t gx = (uint32_t)((a.N + 255) / 256 < 65536 ? (a.N + 255) / 256 : 65536);
  hipLaunchKernelGGL(k_obs_apply<V>, dim3(gx, batch), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename V>
hipError_t launch_gch_lam_adjoint(const GchAdjArgs<V>& a, uint32_t batch, hipStream_t s) {
  const uint64_t pairs = a.N / 2;
  const uint32_t gx = (uint32_t)((pairs + 255) / 256 < 4096 ? (pairs + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_gch_lam_adjoint<V>, dim3(gx, batch), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const double* partial, const double* w, uint32_t n_traj, uint32_t n_tiles,
                              uint32_t n_dot, double* gdot, const uint32_t* dot_param, uint32_t n_params,
                              double* grad, const double* ev, double* E, hipStream_t s) {
  if (n_dot) hipLaunchKernelGGL(k_grad_dot, dim3(n_dot), dim3(256), 0, s, partial, w, n_traj, n_tiles, n_dot, gdot);
  const uint32_t np = n_params ? n_params : 1;
  hipLaunchKernelGGL(k_grad_gather, dim3((np + 255) / 256), dim3(256), 0, s, gdot, dot_param, n_dot, n_params, grad, ev,
                     w, n_traj, E);
  return hipGetLastError();
}

template <typename V>
hipError_t launch_dense_channel(const DenseArgs<V>& a, uint32_t batch, hipStream_t s) {
  hipLaunchKernelGGL(k_rdm<V>, dim3(a.nblk, batch), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_dense_decide<V>, dim3(batch), dim3(64), 0, s, a);
  const uint64_t NB = a.N >> a.nq;
  const uint32_t gx = (uint32_t)((NB + 255) / 256 < 4096 ? (NB + 255) / 256 : 4096);
  hipLaunchKernelGGL((k_dense_apply<V, false>), dim3(gx, batch), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename V>
hipError_t launch_dense_lam_adjoint(const DenseArgs<V>& a, uint32_t batch, hipStream_t s) {
  const uint64_t NB = a.N >> a.nq;
  const uint32_t gx = (uint32_t)((NB + 255) / 256 < 4096 ? (NB + 255) / 256 : 4096);
  hipLaunchKernelGGL((k_dense_apply<V, true>), dim3(gx, batch), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_weighted_sum(const double* w, const double* ev, uint32_t n, double* E, hipStream_t s) {
  hipLaunchKernelGGL(k_weighted_sum, dim3(1), dim3(64), 0, s, w, ev, n, E);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
  uint32_t g = (uint32_t)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
  if (g == 0) g = 1;
  hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

#define PTSBE_INST(V)                                                                                   \
  template hipError_t launch_pass<V>(const PassArgs<V>&, uint32_t, uint32_t, uint32_t, uint32_t, hipStream_t); \
  template hipError_t launch_scan<V>(const ScanArgs<V>&, uint32_t, double*, hipStream_t);                 \
  template hipError_t launch_norm<V>(const ScanArgs<V>&, uint32_t, double*, hipStream_t);                 \
  template hipError_t launch_marginal<V>(const MarginalArgs<V>&, const MrDecideArgs&, uint32_t, hipStream_t); \
  template hipError_t launch_copy_normalised<V>(const V*, V*, const double*, uint64_t, uint32_t, uint32_t,         \
                                                hipStream_t);                                                         \
  template hipError_t launch_expval<V>(const ExpArgs<V>&, const double*, double*, uint32_t, uint32_t, hipStream_t);
PTSBE_INST(float2)
PTSBE_INST(double2)
template hipError_t launch_adjoint_pass<float2>(const AdjArgs<float2>&, uint32_t, uint32_t, uint32_t, hipStream_t);
template hipError_t launch_adjoint_pass<double2>(const AdjArgs<double2>&, uint32_t, uint32_t, uint32_t, hipStream_t);
template hipError_t launch_gch_lam_adjoint<float2>(const GchAdjArgs<float2>&, uint32_t, hipStream_t);
template hipError_t launch_gch_lam_adjoint<double2>(const GchAdjArgs<double2>&, uint32_t, hipStream_t);
template hipError_t launch_obs_apply<float2>(const ObsArgs<float2>&, uint32_t, hipStream_t);
template hipError_t launch_obs_apply<double2>(const ObsArgs<double2>&, uint32_t, hipStream_t);
template hipError_t launch_dense_channel<float2>(const DenseArgs<float2>&, uint32_t, hipStream_t);
template hipError_t launch_dense_channel<double2>(const DenseArgs<double2>&, uint32_t, hipStream_t);
template hipError_t launch_dense_lam_adjoint<float2>(const DenseArgs<float2>&, uint32_t, hipStream_t);
template hipError_t launch_dense_lam_adjoint<double2>(const DenseArgs<double2>&, uint32_t, hipStream_t);
template hipError_t launch_sample<uint32_t>(const SampleArgs<uint32_t>&, uint64_t, hipStream_t);
template hipError_t launch_sample<uint64_t>(const SampleArgs<uint64_t>&, uint64_t, hipStream_t);

}  // namespace ptsbe
