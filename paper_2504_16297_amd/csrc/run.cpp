// Batched execution (Sec. 3, BE): workspace carving, table upload and the
// launch sequence of one ptsbe_run_batch call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "host.hpp"
#include "jit.hpp"
#include "kernels.hpp"

namespace ptsbe {

// Prefix sharing applies to plans whose first pass starts from |0> and whose
// last step is a pass, when at least two trajectories are run and it is not
// off.  Measure-resets may sit between the passes: their outcome is a function
// of the state alone ([p1 > 1/2]), so a trajectory still on the error-free
// prefix takes the prefix state's decisions.  State-dependent channels draw a
// uniform per trajectory and end the sharing for their plans.
bool prefix_sharing(const Plan& P, const TrajSet& ts, const ptsbe_run_opts* o) {
  if (o->flags & PTSBE_RUN_NO_PREFIX_SHARING) return false;
  if (P.n_general || ts.m.size() < 2 || P.exec.empty()) return false;
  for (const ExecStep& ex : P.exec)
    if (ex.dense || ex.restore >= 0) return false;
  if (P.exec.front().pass < 0 || P.exec.back().pass < 0) return false;
  return (P.passes[P.exec[0].pass].flags & PASS_INIT_ZERO) != 0;
}

// Launch routes of one batch under prefix sharing.  eff[b] is the first
// execution step whose pass the trajectory's record changes (the last step,
// a pass, if none does); before it the trajectory's state equals the
// error-free state, which is carried in slots bb and bb + 1 (read one, write
// the other, swap).  At pass step e: trajectories with eff == e read the
// carried state, those with eff < e their own, and the carrier advances while
// some eff > e.  At a measure-reset step e the rows are the states to decide:
// each trajectory with eff < e, and the carried state (destination bb) while
// some eff > e.  eff is appended to eff_out (batch order).
void build_routes(const Plan& P, const TrajSet& ts, uint32_t b0, uint32_t bb, std::vector<uint32_t>& out,
                  std::vector<uint32_t>& off, std::vector<uint32_t>& eff_out) {
  const TableLayout& T = ts.layout;
  const uint32_t* ov_off = reinterpret_cast<const uint32_t*>(ts.table_blob.data() + T.ov_off);
  const uint32_t NP = (uint32_t)P.passes.size();
  const uint32_t E = (uint32_t)P.exec.size();
  std::vector<uint32_t> eff(bb, E - 1);
  for (uint32_t b = 0; b < bb; ++b) {
    const uint64_t row = (uint64_t)(b0 + b) * NP;
    for (uint32_t e = 0; e < E; ++e) {
      if (P.exec[e].pass < 0) continue;
      const uint32_t p = (uint32_t)P.exec[e].pass;
      if (ov_off[row + p + 1] > ov_off[row + p]) {
        eff[b] = e;
        break;
      }
    }
  }
  uint32_t cur = bb, nxt = bb + 1;
  off.assign(E + 1, 0);
  for (uint32_t e = 0; e < E; ++e) {
    off[e] = (uint32_t)(out.size() / 2);
    bool carry = false;
    if (P.exec[e].pass < 0) {
      for (uint32_t b = 0; b < bb; ++b) {
        if (eff[b] < e) {
          out.push_back(b);
          out.push_back(b);
        } else {
          carry = true;
        }
      }
      if (carry) {
        out.push_back(cur);
        out.push_back(bb);
      }
      continue;
    }
    for (uint32_t b = 0; b < bb; ++b) {
      if (eff[b] < e) {
        out.push_back(b);
        out.push_back(b);
      } else if (eff[b] == e) {
        out.push_back(e == 0 ? b : cur);
        out.push_back(b);
      } else {
        carry = true;
      }
    }
    if (carry) {
      out.push_back(cur);
      out.push_back(nxt);
      std::swap(cur, nxt);
    }
  }
  off[E] = (uint32_t)(out.size() / 2);
  eff_out.insert(eff_out.end(), eff.begin(), eff.end());
}

namespace {

uint64_t a256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

struct WsLayout {
  uint64_t status, tables, routes, eff, states, cdf, partial, offs, total, mr_partial, mr_bits, mr_norm, rec_info,
      weights, sup_part, sup_offs, sup_count, sup_cdf, sup_idx, maxa, floor, end;
  bool support;
  uint32_t batch;
  uint32_t nblk, per_block, per_thread;
  bool share;
};

WsLayout layout_for(const Plan& P, const TrajSet& ts, uint32_t mode, uint32_t batch, uint64_t table_bytes,
                    bool share, bool support) {
  WsLayout L{};
  const uint64_t N = 1ull << P.n;
  const uint64_t esz = P.precision == PTSBE_C64 ? 8 : 16;
  const uint64_t Btot = ts.m.size();
  const uint64_t n_batches = (Btot + batch - 1) / std::max<uint32_t>(batch, 1);
  L.batch = batch;
  L.share = share;
  L.per_block = (uint32_t)std::min<uint64_t>(N, kScanBlock);
  L.nblk = (uint32_t)(N / L.per_block);
  L.per_thread = std::max<uint32_t>(1, L.per_block / 256);
  uint64_t o = 0;
  L.status = o; o = a256(o + 16);
  L.tables = o; o = a256(o + table_bytes);
  L.routes = o;
  if (share) o = a256(o + P.exec.size() * (Btot + n_batches) * sizeof(uint2));
  L.eff = o;
  if (share) o = a256(o + Btot * sizeof(uint32_t));
  L.states = o; o = a256(o + (uint64_t)(batch + (share ? 2 : 0)) * N * esz);
  L.cdf = o;
  if (mode == PTSBE_RUN_SHOTS && P.precision == PTSBE_C128) o = a256(o + (uint64_t)batch * N * 8);
  L.partial = o; o = a256(o + (uint64_t)batch * L.nblk * 8);
  L.offs = o; o = a256(o + (uint64_t)batch * L.nblk * 8);
  L.total = o; o = a256(o + (uint64_t)batch * 8);
  L.mr_partial = o;
  if (P.n_measure) o = a256(o + (uint64_t)batch * L.nblk * (kMaxGroup + 1) * 8);
  // records: one row per trajectory, plus the error-free prefix state's row under sharing
  const uint64_t rec_rows = Btot + (share ? 1 : 0);
  L.mr_bits = o; o = a256(o + std::max<uint64_t>(1, rec_rows * P.n_measure));
  L.mr_norm = o; o = a256(o + std::max<uint64_t>(1, rec_rows * P.n_measure) * 8);
  L.rec_info = o;
  if (P.n_general) o = a256(o + (uint64_t)P.n_measure * 8 + P.rec_info.chan_param.size() * 8);
  L.weights = o;
  if (mode == PTSBE_RUN_EXPECTATION) o = a256(o + std::max<uint64_t>(1, Btot) * 8);
  // support lists for the sampler: every block start is in a list, so they can
  // only be short when the state has few blocks
  L.support = support && mode == PTSBE_RUN_SHOTS && L.nblk <= kSupportMax / 2;
  L.sup_part = o;
  if (L.support) o = a256(o + (uint64_t)batch * L.nblk * 8);
  L.sup_offs = o;
  if (L.support) o = a256(o + (uint64_t)batch * L.nblk * 8);
  L.sup_count = o;
  if (L.support) o = a256(o + (uint64_t)batch * 4);
  L.sup_cdf = o;
  if (L.support) o = a256(o + (uint64_t)batch * kSupportMax * 8);
  L.sup_idx = o;
  if (L.support) o = a256(o + (uint64_t)batch * kSupportMax * 8);
  // monotone CDF of the sampler: per (state, block) largest in-block prefix and floor
  L.maxa = o;
  if (mode == PTSBE_RUN_SHOTS) o = a256(o + (uint64_t)batch * L.nblk * 8);
  L.floor = o;
  if (mode == PTSBE_RUN_SHOTS) o = a256(o + (uint64_t)batch * L.nblk * 8);
  L.end = o;
  return L;
}

ptsbe_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return PTSBE_OK;
  return fail(PTSBE_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define CK(expr, what)                                  \
  do {                                                  \
    ptsbe_status _s = hip_check((expr), (what));        \
    if (_s != PTSBE_OK) return _s;                      \
  } while (0)

// Useful FLOPs per amplitude of a pass: 14 per 2x2 matrix (two complex
// products and a sum per output), 30 per 4x4, 6 per diagonal.
// Useful real floating-point operations per amplitude of a pass, on the path
// a block without overrides takes: a 2x2 complex matrix makes each output from
// two complex products and a sum (14); with a real diagonal (phase frame) one
// product is real times complex (10), with a unit diagonal one product and a
// sum (8); a 4x4 costs 30, a diagonal 6, a
// measure-reset 2; slots merged into a phase frame, signs and relabellings 0.
static double m1_flops(const Pass& ps, int slot) {
  switch (ps.slots[slot].frame) {
    case FRAME_REAL_DIAG: return 10;
    case FRAME_UNIT_DIAG: return 8;
    case FRAME_ABSORB:
    case FRAME_OVERRIDE_ONLY: return 0;
    default: return 14;
  }
}

double pass_flops_per_amp(const Pass& ps) {
  double f = 0;
  for (const DOp& op : ps.ops) {
    switch (op.type) {
      case DOP_M1: f += m1_flops(ps, op.slot[0]); break;
      case DOP_M1G:
        for (int j = 0; j < 4; ++j)
          if ((op.mask >> j) & 1) f += m1_flops(ps, op.slot[j]);
        break;
      case DOP_M2: f += ps.slots[op.slot[0]].frame == FRAME_UNIT4 ? 25.5 : 30; break;  // 3 rows of 24, one of 30
      case DOP_D1: f += ps.slots[op.slot[0]].frame == FRAME_ABSORB ? 0 : 6; break;
      case DOP_D2: f += 6; break;
      case DOP_MR: f += 2; break;
      case DOP_KR: f += 14; break;
      default: break;
    }
  }
  return f;
}

// Stage timer: HIP events recorded on the caller's stream between launches;
// the time between two marks is charged to the stage named by the later mark.
struct StageTimer {
  hipStream_t s;
  bool on;
  std::vector<hipEvent_t> ev;
  std::vector<int> cat;
  StageTimer(hipStream_t st, bool enabled) : s(st), on(enabled) {}
  ~StageTimer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  hipError_t mark(int c) {
    if (!on) return hipSuccess;
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    ev.push_back(e);
    cat.push_back(c);
    return hipEventRecord(e, s);
  }
  hipError_t collect(double* out) {
    if (!on || ev.empty()) return hipSuccess;
    hipError_t r = hipEventSynchronize(ev.back());
    if (r != hipSuccess) return r;
    for (size_t i = 1; i < ev.size(); ++i) {
      float ms = 0;
      r = hipEventElapsedTime(&ms, ev[i - 1], ev[i]);
      if (r != hipSuccess) return r;
      if (cat[i] >= 0) out[cat[i]] += ms;
      out[5] += ms;
    }
    return hipSuccess;
  }
};
enum { T_PASS = 0, T_MEASURE = 2, T_SCAN = 3, T_SAMPLE = 4, T_OTHER = -1 };

enum { PH_UPLOAD = 1, PH_LAUNCH = 2 };

}  // namespace

// Arguments of a dense state-dependent channel step (see DenseArgs).
template <typename V>
DenseArgs<V> dense_args(const Plan& P, const ExecStep& ex, V* states, uint8_t* partial, uint8_t* mr_bits,
                        double* mr_norm, uint32_t* status, const double* d_chan_param, uint32_t b0, uint64_t seed,
                        uint32_t cfg, uint64_t alpha0) {
  DenseArgs<V> a{};
  a.swz = P.swizzle ? 1u : 0u;
  a.states = states;
  a.partial = reinterpret_cast<double*>(partial);
  a.N = 1ull << P.n;
  a.nq = (uint32_t)ex.mr_qubits.size();
  for (uint32_t j = 0; j < a.nq; ++j) a.q[j] = (uint32_t)ex.mr_qubits[j];
  a.nblk = (uint32_t)(((a.N >> a.nq) + 4095) / 4096);
  a.mr_bits = mr_bits;
  a.mr_norm = mr_norm;
  a.status = status;
  const uint32_t r = (uint32_t)ex.mr_index[0];
  a.chan = d_chan_param + P.rec_info.rec_chan[r];
  a.rec = r;
  a.gidx = P.rec_info.rec_gidx[r];
  a.n_measure = (uint32_t)P.n_measure;
  a.t0 = b0;
  a.cfg = cfg;
  a.seed = seed;
  a.alpha0 = alpha0;
  return a;
}
template DenseArgs<float2> dense_args<float2>(const Plan&, const ExecStep&, float2*, uint8_t*, uint8_t*, double*,
                                              uint32_t*, const double*, uint32_t, uint64_t, uint32_t, uint64_t);
template DenseArgs<double2> dense_args<double2>(const Plan&, const ExecStep&, double2*, uint8_t*, uint8_t*, double*,
                                                uint32_t*, const double*, uint32_t, uint64_t, uint32_t, uint64_t);

namespace {

// PH_UPLOAD copies the tables and launch routes into the workspace; PH_LAUNCH
// enqueues the kernels (device work only, so it can be captured in a graph).
template <typename V, typename BitT>
ptsbe_status run_typed(const Plan& P, TrajSet& ts, const ptsbe_run_opts& o, uint8_t* ws, const WsLayout& L,
                       void* d_bits, uint32_t* d_traj, uint8_t* d_mr_bits, hipStream_t s, int phase,
                       bool use_jit, uint32_t* d_status) {
  const uint32_t B = (uint32_t)ts.m.size();
  const uint64_t N = 1ull << P.n;
  const TableLayout& T = ts.layout;
  uint8_t* tb = ws + L.tables;
  if (phase & PH_UPLOAD)
    CK(hipMemcpyAsync(tb, ts.table_blob.data(), ts.table_blob.size(), hipMemcpyHostToDevice, s), "table upload");
  // decision data of state-dependent channels (plan-owned host arrays)
  const uint32_t* d_rec_chan = nullptr;
  const uint32_t* d_rec_gidx = nullptr;
  const double* d_chan_param = nullptr;
  if (P.n_general) {
    uint8_t* ri = ws + L.rec_info;
    const size_t nm = (size_t)P.n_measure;
    if (phase & PH_UPLOAD) {
      CK(hipMemcpyAsync(ri, P.rec_info.rec_chan.data(), nm * 4, hipMemcpyHostToDevice, s), "record upload");
      CK(hipMemcpyAsync(ri + nm * 4, P.rec_info.rec_gidx.data(), nm * 4, hipMemcpyHostToDevice, s), "record upload");
      CK(hipMemcpyAsync(ri + nm * 8, P.rec_info.chan_param.data(), P.rec_info.chan_param.size() * 8,
                        hipMemcpyHostToDevice, s), "record upload");
    }
    d_rec_chan = reinterpret_cast<const uint32_t*>(ri);
    d_rec_gidx = reinterpret_cast<const uint32_t*>(ri + nm * 4);
    d_chan_param = reinterpret_cast<const double*>(ri + nm * 8);
  }
  if ((phase & PH_UPLOAD) && o.mode == PTSBE_RUN_EXPECTATION && o.d_ensemble) {
    // the weights stay in the trajectory set until its next run (the copy is asynchronous)
    ts.weights_host = ensemble_weights(ts);
    CK(hipMemcpyAsync(ws + L.weights, ts.weights_host.data(), (size_t)B * 8, hipMemcpyHostToDevice, s),
       "weights upload");
  }
  uint32_t* status = reinterpret_cast<uint32_t*>(ws + L.status);
  if (phase & PH_LAUNCH) CK(launch_fill_u32(status, 0, 4, s), "status reset");
  V* states = reinterpret_cast<V*>(ws + L.states);
  double* partial = reinterpret_cast<double*>(ws + L.partial);
  double* offs = reinterpret_cast<double*>(ws + L.offs);
  double* total = reinterpret_cast<double*>(ws + L.total);
  uint8_t* mr_bits = ws + L.mr_bits;
  double* mr_norm = reinterpret_cast<double*>(ws + L.mr_norm);
  const uint32_t chunk = o.sort_chunk ? o.sort_chunk : 4096;
  const bool timed = o.timing != nullptr && (phase & PH_LAUNCH);
  StageTimer tm(s, timed);
  if (timed)
    for (int i = 0; i < 10; ++i) o.timing[i] = 0.0;
  // routes of every batch, uploaded once
  std::vector<uint32_t>& route_off = ts.route_off;
  std::vector<uint32_t>& routes = ts.route_host;
  std::vector<uint32_t>& eff = ts.eff_host;
  routes.clear();
  route_off.clear();
  eff.clear();
  if (L.share) {
    std::vector<uint32_t> off;
    for (uint32_t b0 = 0; b0 < B; b0 += L.batch) {
      build_routes(P, ts, b0, std::min<uint32_t>(L.batch, B - b0), routes, off, eff);
      route_off.insert(route_off.end(), off.begin(), off.end());
    }
    if (phase & PH_UPLOAD) {
      CK(hipMemcpyAsync(ws + L.routes, routes.data(), routes.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s),
         "route upload");
      if (P.n_measure)
        CK(hipMemcpyAsync(ws + L.eff, eff.data(), eff.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s),
           "route upload");
    }
  }
  if (!(phase & PH_LAUNCH)) return PTSBE_OK;
  const uint2* d_routes = reinterpret_cast<const uint2*>(ws + L.routes);
  const uint32_t* d_eff = reinterpret_cast<const uint32_t*>(ws + L.eff);
  CK(tm.mark(T_OTHER), "timer");

  PassArgs<V> pa{};
  pa.passes = reinterpret_cast<const DPass*>(tb + T.passes);
  pa.ops = reinterpret_cast<const DOp*>(tb + T.ops);
  pa.slot_default = reinterpret_cast<const uint32_t*>(tb + T.slot_default);
  pa.pool = reinterpret_cast<const V*>(tb + T.pool);
  pa.ov_off = reinterpret_cast<const uint32_t*>(tb + T.ov_off);
  pa.ov = reinterpret_cast<const DOverride*>(tb + T.ov);
  pa.mr_bits = mr_bits;
  pa.mr_norm = mr_norm;
  pa.states = states;
  pa.N = N;
  pa.n = (uint32_t)P.n;
  pa.n_passes = (uint32_t)P.passes.size();
  pa.n_measure = (uint32_t)P.n_measure;
  pa.swz = P.swizzle ? 1u : 0u;
  pa.carrier_t = B;  // the record row after the set's last trajectory

  const uint32_t E = (uint32_t)P.exec.size();
  for (uint32_t b0 = 0, bi = 0; b0 < B; b0 += L.batch, ++bi) {
    const uint32_t bb = std::min<uint32_t>(L.batch, B - b0);
    pa.t0 = b0;
    pa.carrier0 = bb;
    for (uint32_t e = 0; e < E; ++e) {
      const ExecStep& ex = P.exec[e];
      if (ex.pass >= 0) {
        const Pass& ps = P.passes[ex.pass];
        pa.pass = (uint32_t)ex.pass;
        uint32_t rows = bb;
        pa.route = nullptr;
        if (L.share) {
          const uint32_t r0 = route_off[(size_t)bi * (E + 1) + e], r1 = route_off[(size_t)bi * (E + 1) + e + 1];
          rows = r1 - r0;
          pa.route = d_routes + r0;
        }
        if (rows && use_jit && jit_has(P, (uint32_t)ex.pass)) {
          CK(jit_launch<V>(P, (uint32_t)ex.pass, pa, rows, s), "compiled tile pass");
        } else if (rows) {
          if (ps.k > 12)  // the generic kernels hold at most 12-qubit tiles
            return fail(PTSBE_E_UNSUPPORTED, "pass " + std::to_string(ex.pass) +
                                                 " has a 13-qubit tile and no compiled kernel loaded here");
          CK(launch_pass<V>(pa, (uint32_t)ps.k, (uint32_t)ps.slots.size(), (uint32_t)ps.ops.size(), rows, s),
             "tile pass");
        }
        CK(tm.mark(T_PASS), "timer");
        if (timed) {
          o.timing[1] += 1;
          o.timing[6] += (double)rows * (double)N * sizeof(V) * ((ps.flags & PASS_INIT_ZERO) ? 1.0 : 2.0);
          o.timing[8] += (double)rows * (double)N * pass_flops_per_amp(ps);
          o.timing[9] += rows;
        }
      } else if (ex.dense) {
        CK(launch_dense_channel<V>(dense_args<V>(P, ex, states, ws + L.mr_partial, mr_bits, mr_norm, status,
                                                 d_chan_param, b0, o.seed, o.cfg, ts.alpha0),
                                   bb, s),
           "state-dependent channel");
        CK(tm.mark(T_MEASURE), "timer");
      } else {
        // states to decide: the batch, or under sharing the trajectories past
        // their first own pass and the error-free prefix state
        uint32_t rows = bb;
        const uint2* d_rows = nullptr;
        if (L.share) {
          const uint32_t r0 = route_off[(size_t)bi * (E + 1) + e], r1 = route_off[(size_t)bi * (E + 1) + e + 1];
          rows = r1 - r0;
          d_rows = d_routes + r0;
        }
        for (size_t g0 = 0; rows && g0 < ex.mr_qubits.size(); g0 += kMaxGroup) {
          size_t g1 = std::min(ex.mr_qubits.size(), g0 + kMaxGroup);
          MarginalArgs<V> ma{};
          ma.swz = pa.swz;
          ma.states = states;
          ma.partial = reinterpret_cast<double*>(ws + L.mr_partial);
          ma.N = N;
          ma.nblk = L.nblk;
          ma.per_block = L.per_block;
          ma.nq = (uint32_t)(g1 - g0);
          MrDecideArgs da{};
          da.partial = ma.partial;
          da.mr_bits = mr_bits;
          da.mr_norm = mr_norm;
          da.status = status;
          da.tol = 1e-6;
          da.nblk = L.nblk;
          da.nq = ma.nq;
          da.t0 = b0;
          da.n_measure = (uint32_t)P.n_measure;
          da.rec_chan = d_rec_chan;
          da.rec_gidx = d_rec_gidx;
          da.chan_param = d_chan_param;
          da.seed = o.seed;
          da.cfg = o.cfg;
          da.alpha0 = ts.alpha0;
          da.carries_norm = g0 == 0 ? 1u : 0u;
          for (size_t j = g0; j < g1; ++j) {
            ma.q[j - g0] = (uint32_t)ex.mr_qubits[j];
            da.idx[j - g0] = (uint32_t)ex.mr_index[j];
          }
          ma.rows = d_rows;
          da.rows = d_rows;
          da.carrier0 = bb;
          da.carrier_t = B;
          da.eff = d_eff;
          da.step = e;
          da.bb = bb;
          CK(launch_marginal<V>(ma, da, rows, s), "measure-reset");
          CK(tm.mark(T_MEASURE), "timer");
        }
      }
    }
    ScanArgs<V> sa{};
    sa.swz = pa.swz;
    sa.states = states;
    sa.partial = partial;
    sa.offs = offs;
    sa.N = N;
    sa.nblk = L.nblk;
    sa.per_block = L.per_block;
    sa.per_thread = L.per_thread;
    if (o.mode == PTSBE_RUN_SHOTS) {
      sa.cdf = P.precision == PTSBE_C128 ? reinterpret_cast<double*>(ws + L.cdf) : nullptr;
      sa.maxa = reinterpret_cast<double*>(ws + L.maxa);
      sa.floor = reinterpret_cast<double*>(ws + L.floor);
      if (L.support) {
        sa.sup_part = reinterpret_cast<double*>(ws + L.sup_part);
        sa.sup_offs = reinterpret_cast<double*>(ws + L.sup_offs);
        sa.sup_count = reinterpret_cast<uint32_t*>(ws + L.sup_count);
        sa.sup_cdf = reinterpret_cast<double*>(ws + L.sup_cdf);
        sa.sup_idx = reinterpret_cast<uint64_t*>(ws + L.sup_idx);
      }
      CK(launch_scan<V>(sa, bb, total, s), "probability scan");
      CK(tm.mark(T_SCAN), "timer");
      SampleArgs<BitT> sm{};
      sm.cdf_base = sa.cdf ? sa.cdf : reinterpret_cast<const double*>(states);
      sm.cdf_stride = sa.cdf ? N : N * sizeof(V) / 8;
      sm.total = total;
      sm.shot_off = reinterpret_cast<const uint64_t*>(tb + T.shot_off);
      sm.chunk_off = reinterpret_cast<const uint64_t*>(tb + T.chunk_off);
      sm.uniforms = o.d_uniforms;
      sm.bits = reinterpret_cast<BitT*>(d_bits);
      sm.traj = d_traj;
      sm.N = N;
      sm.seed = o.seed;
      sm.alpha0 = ts.alpha0;
      sm.b0 = b0;
      sm.b1 = b0 + bb;
      sm.chunk = chunk;
      sm.cfg = o.cfg;
      sm.item0 = ts.chunk_off[b0];
      sm.sup_count = sa.sup_count;
      sm.sup_cdf = sa.sup_cdf;
      sm.sup_idx = sa.sup_idx;
      const uint64_t items = ts.chunk_off[b0 + bb] - ts.chunk_off[b0];
      if (items) {
        CK(launch_sample<BitT>(sm, items, s), "sampler");
        CK(tm.mark(T_SAMPLE), "timer");
        if (timed) o.timing[7] += 1;
      }
    } else if (o.mode == PTSBE_RUN_STATES) {
      CK(launch_norm<V>(sa, bb, total, s), "norm");
      CK(launch_copy_normalised<V>(states, reinterpret_cast<V*>(o.d_state_out) + (uint64_t)b0 * N, total, N, bb, pa.swz, s),
         "state copy");
    } else {
      CK(launch_norm<V>(sa, bb, total, s), "norm");
      ExpArgs<V> ea{};
      ea.swz = pa.swz;
      ea.states = states;
      ea.partial = partial;
      ea.N = N;
      ea.nblk = L.nblk;
      ea.per_block = L.per_block;
      ea.n_terms = o.n_terms;
      for (uint32_t j = 0; j < o.n_terms; ++j) {
        ea.coef[j] = o.obs_coef[j];
        ea.zmask[j] = o.obs_zmask[j];
      }
      CK(launch_expval<V>(ea, total, o.d_expval, bb, b0, s), "expectation");
    }
  }
  if (o.mode == PTSBE_RUN_EXPECTATION && o.d_ensemble)
    CK(launch_weighted_sum(reinterpret_cast<const double*>(ws + L.weights), o.d_expval, B, o.d_ensemble, s),
       "ensemble value");
  if (d_mr_bits && P.n_measure)
    CK(hipMemcpyAsync(d_mr_bits, mr_bits, (size_t)B * P.n_measure, hipMemcpyDeviceToDevice, s), "record copy");
  if (d_status) CK(hipMemcpyAsync(d_status, status, 4, hipMemcpyDeviceToDevice, s), "status copy");
  CK(tm.mark(T_OTHER), "timer");
  if (timed) CK(tm.collect(o.timing), "timer");
  return PTSBE_OK;
}

// `outputs`: also check the output pointers (not needed for a size query)
ptsbe_status check_opts(const Plan& P, const TrajSet& ts, const ptsbe_run_opts* o, bool outputs) {
  if (!o) return fail(PTSBE_E_ARG, "null run options");
  if (o->mode > PTSBE_RUN_EXPECTATION) return fail(PTSBE_E_ARG, "bad run mode");
  uint32_t c = o->sort_chunk ? o->sort_chunk : 4096;
  if (c < 256 || c > 4096 || (c & (c - 1))) return fail(PTSBE_E_ARG, "sort_chunk must be a power of two in 256..4096");
  if (P.n_params && !o->params) return fail(PTSBE_E_ARG, "the circuit has parameters: params required");
  // per-trajectory outputs are needed only when there are trajectories
  const bool any = !ts.m.empty();
  if (outputs && any && o->mode == PTSBE_RUN_STATES && !o->d_state_out)
    return fail(PTSBE_E_ARG, "STATES mode needs d_state_out");
  if (o->mode == PTSBE_RUN_EXPECTATION) {
    if (outputs && any && !o->d_expval) return fail(PTSBE_E_ARG, "EXPECTATION mode needs d_expval");
    if (o->n_terms > 64 || (o->n_terms && (!o->obs_coef || !o->obs_zmask)))
      return fail(PTSBE_E_ARG, "observable: at most 64 Z-string terms with coefficients and masks");
  }
  return PTSBE_OK;
}

}  // namespace

ptsbe_status workspace_size(const Plan& P, TrajSet& ts, const ptsbe_run_opts* o, size_t* bytes) {
  ptsbe_status st = check_opts(P, ts, o, false);
  if (st != PTSBE_OK) return st;
  uint32_t chunk = o->sort_chunk ? o->sort_chunk : 4096;
  {
    std::lock_guard<std::mutex> lk(ts.mu);
    st = build_tables(ts, o->params, chunk);
    if (st != PTSBE_OK) return st;
  }
  uint32_t B = (uint32_t)ts.m.size();
  uint32_t batch = o->max_batch ? std::min<uint32_t>(o->max_batch, std::max<uint32_t>(B, 1)) : std::max<uint32_t>(B, 1);
  batch = std::min<uint32_t>(batch, 65534);
  *bytes = layout_for(P, ts, o->mode, batch, ts.table_blob.size(), prefix_sharing(P, ts, o),
                      !(o->flags & PTSBE_RUN_NO_SUPPORT_LISTS)).end;
  return PTSBE_OK;
}

ptsbe_status run_batch(const Plan& P, TrajSet& ts, const ptsbe_run_opts* o, void* d_ws, size_t ws_bytes,
                       void* d_bits, uint32_t* d_traj, uint64_t capacity, uint8_t* d_mr_bits, void* stream,
                       hipGraphExec_t* graph_out, bool no_alloc, uint32_t* d_status) {
  ptsbe_status st = check_opts(P, ts, o, true);
  if (st != PTSBE_OK) return st;
  if (no_alloc && o->timing) return fail(PTSBE_E_ARG, "timing is not available without allocation (it creates events)");
  if (!d_ws) return fail(PTSBE_E_ARG, "null workspace");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256) return fail(PTSBE_E_ARG, "workspace must be 256-byte aligned");
  if (o->mode == PTSBE_RUN_SHOTS) {
    if (capacity < ts.total_shots) {
      return fail(PTSBE_E_CAPACITY, "output capacity " + std::to_string(capacity) + " < total shots " +
                                        std::to_string(ts.total_shots));
    }
    if (ts.total_shots && (!d_bits || !d_traj)) return fail(PTSBE_E_ARG, "null shot outputs");
  }
  std::lock_guard<std::mutex> lk(ts.mu);
  uint32_t chunk = o->sort_chunk ? o->sort_chunk : 4096;
  st = build_tables(ts, o->params, chunk);
  if (st != PTSBE_OK) return st;
  const uint32_t B = (uint32_t)ts.m.size();
  if (B == 0) {
    // nothing to prepare or draw (an ensemble value or a graph would be
    // undefined); the status word is cleared so that ptsbe_run_status reads OK
    if (graph_out) return fail(PTSBE_E_ARG, "empty trajectory set: nothing to capture");
    if (o->mode == PTSBE_RUN_EXPECTATION && o->d_ensemble)
      return fail(PTSBE_E_ARG, "empty trajectory set: the ensemble value has no weights");
    if (ws_bytes < 16) return fail(PTSBE_E_ARG, "workspace smaller than its 16-byte status word");
    hipStream_t s0 = static_cast<hipStream_t>(stream);
    CK(launch_fill_u32(static_cast<uint32_t*>(d_ws), 0, 4, s0), "status reset");
    if (d_status) CK(launch_fill_u32(d_status, 0, 1, s0), "status reset");
    return PTSBE_OK;
  }
  uint32_t batch = o->max_batch ? std::min(o->max_batch, B) : B;
  batch = std::min<uint32_t>(batch, 65534);  // grid.y limit of the per-state launches (+1 carrier row)
  const bool share = prefix_sharing(P, ts, o);
  const bool support = !(o->flags & PTSBE_RUN_NO_SUPPORT_LISTS);
  WsLayout L = layout_for(P, ts, o->mode, batch, ts.table_blob.size(), share, support);
  while (L.end > ws_bytes && batch > 1) {
    batch = std::max<uint32_t>(1, batch / 2);
    L = layout_for(P, ts, o->mode, batch, ts.table_blob.size(), share, support);
  }
  if (L.end > ws_bytes)
    return fail(PTSBE_E_OOM, "workspace of " + std::to_string(ws_bytes) + " bytes is below the " +
                                 std::to_string(L.end) + " bytes needed for one trajectory");
  // Without allocation the compiled passes run only if their code objects are
  // already loaded on this device (loading a module allocates device memory);
  // otherwise the generic tile kernels run the same tables.
  bool use_jit = P.use_jit;
  if (use_jit && !no_alloc) {
    st = jit_build(P);
    if (st != PTSBE_OK) return st;
  }
  if (use_jit && no_alloc) use_jit = jit_loaded(P);
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto dispatch = [&](int phase) -> ptsbe_status {
    if (P.precision == PTSBE_C64) {
      if (P.n <= 32) return run_typed<float2, uint32_t>(P, ts, *o, ws, L, d_bits, d_traj, d_mr_bits, s, phase,
                                                        use_jit, d_status);
      return run_typed<float2, uint64_t>(P, ts, *o, ws, L, d_bits, d_traj, d_mr_bits, s, phase,
                                                        use_jit, d_status);
    }
    if (P.n <= 32) return run_typed<double2, uint32_t>(P, ts, *o, ws, L, d_bits, d_traj, d_mr_bits, s, phase,
                                                        use_jit, d_status);
    return run_typed<double2, uint64_t>(P, ts, *o, ws, L, d_bits, d_traj, d_mr_bits, s, phase,
                                                        use_jit, d_status);
  };
  if (!graph_out) return dispatch(PH_UPLOAD | PH_LAUNCH);
  // graph: upload now, load the compiled kernels, then capture the device work
  if (!s) return fail(PTSBE_E_ARG, "graph capture needs a created stream, not the default stream");
  if (o->timing) return fail(PTSBE_E_ARG, "timing is not available for captured runs");
  st = dispatch(PH_UPLOAD);
  if (st != PTSBE_OK) return st;
  CK(hipStreamSynchronize(s), "table upload");
  CK(jit_load(P), "compiled pass load");
  CK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
  st = dispatch(PH_LAUNCH);
  hipGraph_t g = nullptr;
  hipError_t ce = hipStreamEndCapture(s, &g);
  if (st != PTSBE_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  CK(ce, "end capture");
  hipError_t ie = hipGraphInstantiate(graph_out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  CK(ie, "graph instantiate");
  return PTSBE_OK;
}

ptsbe_status run_status(const void* d_ws, void* stream) {
  if (!d_ws) return fail(PTSBE_E_ARG, "null workspace");
  hipStream_t s = static_cast<hipStream_t>(stream);
  CK(hipStreamSynchronize(s), "stream synchronize");
  uint32_t v = 0;
  CK(hipMemcpy(&v, d_ws, 4, hipMemcpyDeviceToHost), "status read");
  if (v & 1u) return fail(PTSBE_E_NONDET_MEASURE, "a measure-reset outcome was not deterministic (min(p1, 1-p1) > 1e-6)");
  if (v & 2u) return fail(PTSBE_E_DEVICE, "a decision step met a state of zero or non-finite norm");
  return PTSBE_OK;
}

}  // namespace ptsbe
