// Distinct shots per trajectory and the shots compressed to (basis index,
// count) pairs.  Sec. 4 measures, next to the shot rate, the fraction of a
// trajectory's shots that are distinct; this turns the sampler's output into
// that number and into a compressed record of the same shots.
//
// Per batch of trajectories (their shots contiguous in the shot buffer):
//   k_uq_fill    clears one open-addressing hash table per trajectory
//                (capacity a power of two >= 2 min(m, 2^n), so a free slot
//                always exists and every probe sequence ends);
//   k_uq_insert  one thread per shot: linear probing with a 64-bit CAS on the
//                key, then count += 1 and first = min(first, shot's position);
//   k_uq_flag    a shot is its value's first occurrence when first equals its
//                position; per-block sums of those flags;
//   k_uq_scan    exclusive scan of the block sums (one workgroup);
//   k_uq_seg     per trajectory, the scan at its first and one-past-last shot:
//                their difference is its distinct count;
//   k_uq_emit    each first occurrence writes (value, count) at its rank among
//                the trajectory's first occurrences: pairs come out in order of
//                first appearance in the shot stream, so the output does not
//                depend on the order in which threads won their slots.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "host.hpp"

namespace ptsbe {

namespace {

constexpr uint64_t kEmpty = ~0ull;  // no basis index reaches 2^64 - 1
constexpr uint32_t kBlock = 256;

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  // SplitMix64 finaliser (Steele, Lea and Flood, 2014)
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}

struct UqArgs {
  const void* bits;        // shots of the batch start at bits[shot_off[0]] (global shot index)
  uint32_t bit_bytes;      // 4 or 8
  const uint64_t* shot_off;  // nb + 1 global shot offsets of the batch's trajectories
  const uint64_t* tab_off;   // nb + 1 slot offsets of their tables
  uint32_t nb;
  uint64_t s0, ns;         // first global shot of the batch, shots in the batch
  uint64_t* keys;
  uint32_t* cnt;
  uint32_t* first;
  uint32_t* flag;          // ns
  uint64_t* part;          // nblk block sums, then their exclusive scan; part[nblk] = total
  uint64_t* uniq;          // distinct counts of the batch's trajectories (global array + b0)
  uint64_t* seg;           // nb: first occurrences before each trajectory's first shot
  void* out_index;         // optional, same width as bits, indexed like the shots
  uint32_t* out_count;     // optional
};

__device__ __forceinline__ uint64_t load_bit(const UqArgs& a, uint64_t g) {
  return a.bit_bytes == 8 ? reinterpret_cast<const uint64_t*>(a.bits)[g]
                          : (uint64_t) reinterpret_cast<const uint32_t*>(a.bits)[g];
}

// trajectory (batch-relative) of global shot g: shot_off[t] <= g < shot_off[t + 1]
__device__ __forceinline__ uint32_t traj_of(const UqArgs& a, uint64_t g) {
  uint32_t lo = 0, hi = a.nb;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a.shot_off[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

// slot of `key` in trajectory t's table (the key is present)
__device__ __forceinline__ uint64_t find_slot(const UqArgs& a, uint32_t t, uint64_t key) {
  const uint64_t base = a.tab_off[t], H = a.tab_off[t + 1] - base;
  uint64_t s = mix64(key) & (H - 1);
  for (uint64_t probe = 0; probe < H; ++probe) {
    if (a.keys[base + s] == key) return base + s;
    s = (s + 1) & (H - 1);
  }
  return kEmpty;
}

__global__ __launch_bounds__(kBlock) void k_uq_fill(uint64_t* keys, uint32_t* cnt, uint32_t* first, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    keys[i] = kEmpty;
    cnt[i] = 0u;
    first[i] = 0xffffffffu;
  }
}

__global__ __launch_bounds__(kBlock) void k_uq_insert(UqArgs a) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.ns) return;
  const uint64_t g = a.s0 + i;
  const uint32_t t = traj_of(a, g);
  const uint64_t key = load_bit(a, g);
  const uint32_t pos = (uint32_t)(g - a.shot_off[t]);
  const uint64_t base = a.tab_off[t], H = a.tab_off[t + 1] - base;
  uint64_t s = mix64(key) & (H - 1);
  for (uint64_t probe = 0; probe < H; ++probe) {
    unsigned long long* kp = reinterpret_cast<unsigned long long*>(a.keys + base + s);
    const unsigned long long prev = atomicCAS(kp, (unsigned long long)kEmpty, (unsigned long long)key);
    if (prev == kEmpty || prev == key) {
      atomicAdd(a.cnt + base + s, 1u);
      atomicMin(a.first + base + s, pos);
      return;
    }
    s = (s + 1) & (H - 1);
  }
}

__device__ __forceinline__ uint64_t block_excl_scan_u64(uint64_t v, uint64_t* total) {
  __shared__ uint64_t sh[kBlock];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (uint32_t d = 1; d < kBlock; d <<= 1) {
    const uint64_t add = threadIdx.x >= d ? sh[threadIdx.x - d] : 0ull;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  const uint64_t incl = sh[threadIdx.x];
  *total = sh[kBlock - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kBlock) void k_uq_flag(UqArgs a) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t f = 0;
  if (i < a.ns) {
    const uint64_t g = a.s0 + i;
    const uint32_t t = traj_of(a, g);
    const uint64_t slot = find_slot(a, t, load_bit(a, g));
    f = (slot != kEmpty && a.first[slot] == (uint32_t)(g - a.shot_off[t])) ? 1u : 0u;
    a.flag[i] = f;
  }
  uint64_t tot;
  block_excl_scan_u64(f, &tot);
  if (threadIdx.x == 0) a.part[blockIdx.x] = tot;
}

// exclusive scan of the nblk block sums in place; part[nblk] = the total
__global__ __launch_bounds__(kBlock) void k_uq_scan(uint64_t* part, uint32_t nblk) {
  uint64_t carry = 0;
  for (uint32_t b0 = 0; b0 < nblk; b0 += kBlock) {
    const uint32_t b = b0 + threadIdx.x;
    const uint64_t v = b < nblk ? part[b] : 0ull;
    uint64_t tot;
    const uint64_t ex = block_excl_scan_u64(v, &tot);
    if (b < nblk) part[b] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) part[nblk] = carry;
}

// first occurrences among the batch's shots [0, j)
__device__ __forceinline__ uint64_t flags_before(const UqArgs& a, uint64_t j) {
  if (j >= a.ns) return a.part[(a.ns + kBlock - 1) / kBlock];
  const uint64_t blk = j / kBlock;
  uint64_t e = a.part[blk];
  for (uint64_t k = blk * kBlock; k < j; ++k) e += a.flag[k];
  return e;
}

// one thread per trajectory of the batch: its distinct count and where its
// first occurrences start in the batch's rank order
__global__ __launch_bounds__(kBlock) void k_uq_seg(UqArgs a) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.nb) return;
  const uint64_t e0 = flags_before(a, a.shot_off[t] - a.s0), e1 = flags_before(a, a.shot_off[t + 1] - a.s0);
  a.seg[t] = e0;
  a.uniq[t] = e1 - e0;
}

__global__ __launch_bounds__(kBlock) void k_uq_emit(UqArgs a) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t f = i < a.ns ? a.flag[i] : 0u;
  uint64_t tot;
  const uint64_t ex = block_excl_scan_u64(f, &tot);
  if (!f) return;
  const uint64_t g = a.s0 + i;
  const uint32_t t = traj_of(a, g);
  const uint64_t key = load_bit(a, g);
  const uint64_t slot = find_slot(a, t, key);
  if (slot == kEmpty) return;  // not reached: every shot's value was inserted
  const uint64_t rank = a.part[blockIdx.x] + ex - a.seg[t];
  const uint64_t o = a.shot_off[t] + rank;
  if (a.out_index) {
    if (a.bit_bytes == 8) reinterpret_cast<uint64_t*>(a.out_index)[o] = key;
    else reinterpret_cast<uint32_t*>(a.out_index)[o] = (uint32_t)key;
  }
  if (a.out_count) a.out_count[o] = a.cnt[slot];
}

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

uint64_t table_slots(uint64_t m, int n) {
  const uint64_t d = n >= 62 ? m : std::min<uint64_t>(m, 1ull << n);
  uint64_t c = 2;
  while (c < 2 * d) c <<= 1;
  return c;
}

// Workspace of a batch of nb trajectories with `slots` table slots and `shots`
// shots in all: shot and table offsets, tables, flags, block sums, batch scans.
struct UqLayout {
  uint64_t shot_off, tab_off, keys, cnt, first, flag, part, seg, total;
  uint64_t slots, shots, nblk;
};

UqLayout uq_layout(uint64_t nb, uint64_t slots, uint64_t shots) {
  UqLayout L{};
  L.slots = slots;
  L.shots = shots;
  L.nblk = std::max<uint64_t>(1, (shots + kBlock - 1) / kBlock);
  uint64_t o = 0;
  L.shot_off = o; o = align256(o + (nb + 1) * 8);
  L.tab_off = o;  o = align256(o + (nb + 1) * 8);
  L.keys = o;     o = align256(o + slots * 8);
  L.cnt = o;      o = align256(o + slots * 4);
  L.first = o;    o = align256(o + slots * 4);
  L.flag = o;     o = align256(o + std::max<uint64_t>(1, shots) * 4);
  L.part = o;     o = align256(o + (L.nblk + 1) * 8);
  L.seg = o;      o = align256(o + std::max<uint64_t>(1, nb) * 8);
  L.total = o;
  return L;
}

// prefix sums of table slots and shots over the trajectories
struct UqPrefix {
  std::vector<uint64_t> slots, shots;
  UqLayout window(uint32_t b0, uint32_t b1) const {
    return uq_layout(b1 - b0, slots[b1] - slots[b0], shots[b1] - shots[b0]);
  }
};

UqPrefix uq_prefix(const TrajSet& ts) {
  const uint32_t B = (uint32_t)ts.m.size();
  UqPrefix P;
  P.slots.assign(B + 1, 0);
  P.shots.assign(B + 1, 0);
  for (uint32_t t = 0; t < B; ++t) {
    P.slots[t + 1] = P.slots[t] + table_slots(ts.m[t], ts.plan->n);
    P.shots[t + 1] = P.shots[t] + ts.m[t];
  }
  return P;
}

ptsbe_status ck(hipError_t e, const char* what) {
  if (e == hipSuccess) return PTSBE_OK;
  return fail(PTSBE_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

ptsbe_status unique_workspace_size(const TrajSet& ts, uint32_t max_batch, size_t* bytes) {
  const uint32_t B = (uint32_t)ts.m.size();
  const UqPrefix P = uq_prefix(ts);
  const uint32_t w = (max_batch && max_batch < B) ? max_batch : B;
  uint64_t best = P.window(0, w).total;
  for (uint32_t b = 1; b + w <= B; ++b) best = std::max(best, P.window(b, b + w).total);
  *bytes = (size_t)best;
  return PTSBE_OK;
}

ptsbe_status unique_shots(TrajSet& ts, const void* d_bits, void* d_ws, size_t ws_bytes, uint64_t* d_unique,
                          void* d_pair_index, uint32_t* d_pair_count, hipStream_t s) {
  const uint32_t B = (uint32_t)ts.m.size();
  const int n = ts.plan->n;
  if (!d_unique) return fail(PTSBE_E_ARG, "null distinct-count output");
  if (B && ts.total_shots && !d_bits) return fail(PTSBE_E_ARG, "null shot buffer");
  if (!d_ws && ws_bytes) return fail(PTSBE_E_ARG, "null workspace");
  if (reinterpret_cast<uintptr_t>(d_ws) & 255) return fail(PTSBE_E_ARG, "workspace must be 256-byte aligned");
  for (uint32_t t = 0; t < B; ++t)
    if (ts.m[t] > 0xffffffffull) return fail(PTSBE_E_UNSUPPORTED, "more than 2^32 - 1 shots in one trajectory");
  const UqPrefix P = uq_prefix(ts);
  const std::vector<uint64_t>& shot_off = P.shots;
  uint8_t* ws = reinterpret_cast<uint8_t*>(d_ws);
  // host staging of the batches' offset arrays, kept in the trajectory set so
  // that it outlives the asynchronous uploads
  std::vector<uint64_t>& stage = ts.uq_host;
  stage.clear();
  stage.reserve(4 * (size_t)B + 4);
  uint32_t b0 = 0;
  while (b0 < B) {
    // the largest batch from b0 that fits the workspace
    uint32_t b1 = b0 + 1;
    if (P.window(b0, b1).total > ws_bytes)
      return fail(PTSBE_E_ARG, "workspace too small for trajectory " + std::to_string(b0) +
                                   " (see ptsbe_unique_workspace_size)");
    while (b1 < B && P.window(b0, b1 + 1).total <= ws_bytes) ++b1;
    const UqLayout L = P.window(b0, b1);
    const uint32_t nb = b1 - b0;
    const size_t so = stage.size();
    for (uint32_t j = 0; j <= nb; ++j) stage.push_back(shot_off[b0 + j]);
    const size_t to = stage.size();
    for (uint32_t j = 0; j <= nb; ++j) stage.push_back(P.slots[b0 + j] - P.slots[b0]);
    ptsbe_status st;
    if ((st = ck(hipMemcpyAsync(ws + L.shot_off, stage.data() + so, (nb + 1) * 8, hipMemcpyHostToDevice, s),
                 "upload")))
      return st;
    if ((st = ck(hipMemcpyAsync(ws + L.tab_off, stage.data() + to, (nb + 1) * 8, hipMemcpyHostToDevice, s),
                 "upload")))
      return st;
    UqArgs a{};
    a.bits = d_bits;
    a.bit_bytes = n > 32 ? 8u : 4u;
    a.shot_off = reinterpret_cast<const uint64_t*>(ws + L.shot_off);
    a.tab_off = reinterpret_cast<const uint64_t*>(ws + L.tab_off);
    a.nb = nb;
    a.s0 = shot_off[b0];
    a.ns = L.shots;
    a.keys = reinterpret_cast<uint64_t*>(ws + L.keys);
    a.cnt = reinterpret_cast<uint32_t*>(ws + L.cnt);
    a.first = reinterpret_cast<uint32_t*>(ws + L.first);
    a.flag = reinterpret_cast<uint32_t*>(ws + L.flag);
    a.part = reinterpret_cast<uint64_t*>(ws + L.part);
    a.uniq = d_unique + b0;
    a.seg = reinterpret_cast<uint64_t*>(ws + L.seg);
    a.out_index = d_pair_index;
    a.out_count = d_pair_count;
    const uint32_t gfill = (uint32_t)std::min<uint64_t>(4096, (L.slots + kBlock - 1) / kBlock);
    const uint32_t g = (uint32_t)L.nblk;
    if (L.slots)
      hipLaunchKernelGGL(k_uq_fill, dim3(std::max(gfill, 1u)), dim3(kBlock), 0, s, a.keys, a.cnt, a.first, L.slots);
    if (L.shots) hipLaunchKernelGGL(k_uq_insert, dim3(g), dim3(kBlock), 0, s, a);
    // with no shots the flag pass still writes the (zero) block sum the scan reads
    hipLaunchKernelGGL(k_uq_flag, dim3(g), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_uq_scan, dim3(1), dim3(kBlock), 0, s, a.part, g);
    hipLaunchKernelGGL(k_uq_seg, dim3((nb + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
    if (L.shots && (d_pair_index || d_pair_count)) hipLaunchKernelGGL(k_uq_emit, dim3(g), dim3(kBlock), 0, s, a);
    if ((st = ck(hipGetLastError(), "distinct-shot kernels"))) return st;
    b0 = b1;
  }
  return PTSBE_OK;
}

}  // namespace ptsbe
