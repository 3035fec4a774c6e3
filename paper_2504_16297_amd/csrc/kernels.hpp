// Kernel argument blocks and launchers of the gfx950 hot path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tables.hpp"

namespace ptsbe {

constexpr int kMaxGroup = 16;   // measure-resets measured together
constexpr uint32_t kScanBlock = 4096;

// Storage layout of the states.  Amplitude x is stored at position
// swizzle(x) = x ^ (f(x >> 12) << 4): the bits of x from 12 up, mapped to 8 bits
// by a fixed GF(2)-linear f (bit i contributes kSwizzle[i]), are XORed onto
// bits 4..11.  Runs of 16 amplitudes stay contiguous and every 4096-amplitude
// block stays in place (permuted inside), but a tile whose qubits are high
// ones no longer sends its 128-byte runs to addresses that differ only in
// high bits (which measured slower on the HBM: 4.0 against 5.2 TB/s for the
// tile of qubits 0-3 and 20-27 of a 28-qubit state, 4.8 against 5.2 averaged
// over a 28-qubit plan's tiles).  An involution: the same map takes a
// position back to its amplitude.  States below 2^13 amplitudes are unchanged.
constexpr uint32_t kSwizzle[24] = {0x7a, 0x96, 0x3d, 0x72, 0x37, 0xf0, 0x85, 0x96, 0x92, 0xce, 0x15, 0x7a,
                                   0xaf, 0xa8, 0x5d, 0x0e, 0xaa, 0x06, 0xed, 0x62, 0x47, 0x60, 0x35, 0x86};

__host__ __device__ inline uint32_t swizzle_f(uint64_t h) {
  uint32_t f = 0;
#pragma unroll
  for (int i = 0; i < 24; ++i)
    if ((h >> i) & 1u) f ^= kSwizzle[i];
  return f;
}
// The XOR a 4096-amplitude block applies to its in-block offsets (0 when off).
__host__ __device__ inline uint32_t swizzle_block(uint64_t block, uint32_t on) {
  return on ? swizzle_f(block) << 4 : 0u;
}
__host__ __device__ inline uint64_t swizzle(uint64_t x, uint32_t on) {
  return on ? x ^ ((uint64_t)swizzle_f(x >> 12) << 4) : x;
}

// Arguments of one tile-pass launch.  The field list is a macro so that the
// pass compiler can emit the identical structure into the kernels it builds:
//   passes, ops, slot_default, pool, ov_off, ov   device tables (slot_default is
//       pass-local for compiled pass kernels);
//   mr_bits, mr_norm   measure-reset records and renormalisation factors;
//   states             batch of states, state b at states + b * N;
//   route, carrier0    optional routing of block row y: state slot route[y].x is
//       read and slot route[y].y written; slots >= carrier0 hold error-free
//       prefix states and use no overrides, any other slot b is trajectory
//       t0 + b; route == nullptr means y -> y;
//   N, n, pass, n_passes, t0, n_measure, swz;
//   carrier_t          record row (measure-reset bits and factors) of the
//       error-free prefix state (the row after the set's last trajectory).
#define PTSBE_PASS_ARGS_FIELDS(V, DPASS, DOP, DOV, U2)                                        \
  const DPASS* passes;                                                                       \
  const DOP* ops;                                                                            \
  const uint32_t* slot_default;                                                              \
  const V* pool;                                                                             \
  const uint32_t* ov_off;                                                                    \
  const DOV* ov;                                                                             \
  const uint8_t* mr_bits;                                                                    \
  const double* mr_norm;                                                                     \
  V* states;                                                                                 \
  const U2* route;                                                                           \
  uint32_t carrier0;                                                                         \
  uint64_t N;                                                                                \
  uint32_t n;                                                                                \
  uint32_t pass;                                                                             \
  uint32_t n_passes;                                                                         \
  uint32_t t0;                                                                               \
  uint32_t n_measure;                                                                        \
  uint32_t swz;                                                                              \
  uint32_t carrier_t;

template <typename V>
struct PassArgs {
  PTSBE_PASS_ARGS_FIELDS(V, DPass, DOp, DOverride, uint2)
};

// Support lists: the basis indices of a state with |psi_x|^2 > 0 (a superset of
// the indices an upper-bound search of the CDF can return) and their CDF
// values, kept per trajectory when there are at most kSupportMax of them.
constexpr uint32_t kSupportMax = 1024;

template <typename V>
struct ScanArgs {
  V* states;
  double* cdf;      // nullptr: write the CDF in place over complex64 slots
  double* partial;  // batch x nblk
  double* offs;     // batch x nblk
  uint64_t N;
  uint32_t nblk;
  uint32_t per_block;
  uint32_t per_thread;
  uint32_t swz;         // states stored swizzled (see swizzle())
  // monotone CDF (nullptr: plain block scan): per (state, block) its largest
  // in-block prefix and the largest CDF value of the blocks before it
  double* maxa;         // batch x nblk
  double* floor;        // batch x nblk
  // optional support lists (nullptr: none): per (state, block) counts and their
  // exclusive prefix, per state the count, then up to kSupportMax (CDF, index)
  double* sup_part;     // batch x nblk
  double* sup_offs;     // batch x nblk
  uint32_t* sup_count;  // batch
  double* sup_cdf;      // batch x kSupportMax
  uint64_t* sup_idx;    // batch x kSupportMax
};

template <typename V>
struct MarginalArgs {
  uint32_t swz;
  const V* states;
  double* partial;  // batch x nblk x (kMaxGroup + 1)
  uint64_t N;
  uint32_t nblk;
  uint32_t per_block;
  uint32_t nq;
  uint32_t q[kMaxGroup];
  // optional list of the states to sum: row y sums state slot rows[y].x
  // (nullptr: row y sums slot y)
  const uint2* rows;
};

struct MrDecideArgs {
  const double* partial;
  uint8_t* mr_bits;
  double* mr_norm;
  uint32_t* status;
  double tol;
  uint32_t nblk;
  uint32_t nq;
  uint32_t t0;
  uint32_t n_measure;
  uint32_t idx[kMaxGroup];
  // state-dependent channels among the record entries (null if the plan has none)
  const uint32_t* rec_chan;   // per record entry: offset into chan_param, or 0xffffffff (measure-reset)
  const uint32_t* rec_gidx;   // per record entry: word of its uniform
  const double* chan_param;   // per channel: K, d0[0..K), d1[0..K)
  uint64_t seed, alpha0;
  uint32_t cfg;
  // 1 for the first group of a decision step: its first entry also carries the
  // 1/||psi|| renormalisation (a step with more than kMaxGroup entries is
  // decided in several groups from the same state, which is rescaled once)
  uint32_t carries_norm;
  // Prefix sharing (measure-resets only; nullptr: row tb decides trajectory
  // t0 + tb): row tb decides the state of rows[tb] as in MarginalArgs, whose
  // record row is t0 + rows[tb].y, or carrier_t when rows[tb].y >= carrier0
  // (the error-free prefix state).  A second launch copies that row's
  // decisions to every batch trajectory b < bb with eff[t0 + b] > step (still
  // on the prefix).
  const uint2* rows;
  uint32_t carrier0, carrier_t;
  const uint32_t* eff;
  uint32_t step, bb;
};

template <typename BitT>
struct SampleArgs {
  const double* cdf_base;   // CDF of batch state 0
  uint64_t cdf_stride;      // elements between consecutive states' CDFs
  const double* total;      // batch x 1
  const uint64_t* shot_off; // set-local prefix of m
  const uint64_t* chunk_off;
  const double* uniforms;   // optional
  BitT* bits;
  uint32_t* traj;
  uint64_t N;
  uint64_t seed;
  uint64_t alpha0;
  uint64_t item0;
  uint32_t b0, b1;          // trajectories of this batch (set-local)
  uint32_t chunk;
  uint32_t cfg;
  // support lists of the batch's states (nullptr: search the full CDF)
  const uint32_t* sup_count;
  const double* sup_cdf;
  const uint64_t* sup_idx;
};

template <typename V>
struct ExpArgs {
  uint32_t swz;
  const V* states;
  double* partial;
  uint64_t N;
  uint32_t nblk;
  uint32_t per_block;
  uint32_t n_terms;
  double coef[64];
  uint64_t zmask[64];
};

// Reverse sweep of the adjoint gradient: psi and lambda tiles in LDS, every op
// applied to both, DOT ops write Im<lambda|P|psi> partials per (trajectory, tile).
template <typename V>
struct AdjArgs {
  PassArgs<V> p;        // tables of the adjoint program; p.states = psi
  V* lam;               // lambda states (same layout as psi)
  double* partial;      // [trajectory][tile][dot]
  uint32_t n_dot;
};

template <typename V>
struct ObsArgs {
  uint32_t swz;
  const V* psi;
  V* lam;
  uint64_t N;
  uint32_t n_terms;
  double coef[64];
  uint64_t zmask[64];
};

// Reverse sweep at a state-dependent channel on qubit q: lambda <- G^dagger
// lambda for the operator G = s K_k the forward sweep applied (k and s from
// record entry `rec` of each trajectory, K_k from the channel's parameters).
template <typename V>
struct GchAdjArgs {
  uint32_t swz;
  V* lam;
  const uint8_t* mr_bits;
  const double* mr_norm;
  const double* chan;   // the channel's block of the record data: K, d0[K], d1[K], K x 8 operator doubles
  uint64_t N;
  uint32_t q;
  uint32_t rec;
  uint32_t n_measure;
  uint32_t t0;
};

// A dense state-dependent channel on qubits q[0..nq-1] (nq 1 or 2; bit j of a
// Kraus matrix index <-> q[j]), for every state of the batch: the reduced
// density matrix rho of those qubits in FP64 (per-block partial sums, reduced
// in a fixed order), p_k = Re Tr(M_k rho) / Tr rho with M_k = K_k^dagger K_k,
// k drawn with the uniform of word gidx of the stream [seed, 4<<56 | cfg<<48 |
// alpha] (smallest k with u < p_0 + ... + p_k over p_k > 0, else the last such
// k), recorded with the factor 1 / sqrt(p_k Tr rho), and K_k times that factor
// applied to the state.  chan: K, d, then M_k and K_k for every k (d x d
// row-major complex, re/im interleaved).
template <typename V>
struct DenseArgs {
  uint32_t swz;
  V* states;
  double* partial;      // batch x nblk x 16
  uint64_t N;
  uint32_t nq;
  uint32_t q[2];
  uint32_t nblk;        // blocks of 4096 base indices (indices with the channel's qubits 0)
  uint8_t* mr_bits;
  double* mr_norm;
  uint32_t* status;
  const double* chan;
  uint32_t rec, gidx, n_measure, t0, cfg;
  uint64_t seed, alpha0;
  V* lam;               // reverse sweep: lambda <- (factor K_k)^dagger lambda
};
template <typename V>
hipError_t launch_dense_channel(const DenseArgs<V>& a, uint32_t batch, hipStream_t s);
template <typename V>
hipError_t launch_dense_lam_adjoint(const DenseArgs<V>& a, uint32_t batch, hipStream_t s);

template <typename V>
hipError_t launch_adjoint_pass(const AdjArgs<V>& a, uint32_t k, uint32_t n_slots, uint32_t batch, hipStream_t s);
template <typename V>
hipError_t launch_gch_lam_adjoint(const GchAdjArgs<V>& a, uint32_t batch, hipStream_t s);
template <typename V>
hipError_t launch_obs_apply(const ObsArgs<V>& a, uint32_t batch, hipStream_t s);
// gdot[d] = sum_t w[t] sum_tile partial[t][tile][d]; grad[p] = sum over dots of p; E = sum_t w[t] ev[t]
hipError_t launch_grad_reduce(const double* partial, const double* w, uint32_t n_traj, uint32_t n_tiles,
                              uint32_t n_dot, double* gdot, const uint32_t* dot_param, uint32_t n_params,
                              double* grad, const double* ev, double* E, hipStream_t s);

template <typename V>
hipError_t launch_pass(const PassArgs<V>& a, uint32_t k, uint32_t n_slots, uint32_t n_ops, uint32_t batch,
                       hipStream_t s);
template <typename V>
hipError_t launch_scan(const ScanArgs<V>& a, uint32_t batch, double* total, hipStream_t s);
template <typename V>
hipError_t launch_norm(const ScanArgs<V>& a, uint32_t batch, double* total, hipStream_t s);
template <typename V>
hipError_t launch_marginal(const MarginalArgs<V>& a, const MrDecideArgs& d, uint32_t batch, hipStream_t s);
template <typename BitT>
hipError_t launch_sample(const SampleArgs<BitT>& a, uint64_t items, hipStream_t s);
template <typename V>
hipError_t launch_copy_normalised(const V* states, V* out, const double* total, uint64_t N, uint32_t batch,
                                  uint32_t swz, hipStream_t s);
template <typename V>
hipError_t launch_expval(const ExpArgs<V>& a, const double* total, double* out, uint32_t batch, uint32_t t0,
                         hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
hipError_t launch_weighted_sum(const double* w, const double* ev, uint32_t n, double* E, hipStream_t s);

}  // namespace ptsbe
