// Adjoint gradient of the probability-weighted trajectory ensemble.
//
// Pre-trajectory sampling fixes every trajectory's Kraus operators before
// execution (Sec. 3), so each trajectory is a fixed unitary circuit U_a(theta)
// and E(theta) = sum_a w_a <psi_a|O|psi_a>, with w_a = count_a / sum count
// independent of theta for unitary-mixture noise.  Per trajectory: psi = U|0>
// (forward program), lambda = O psi, then the reverse-sweep program un-applies
// every operation on psi and lambda and, just before un-applying a rotation
// exp(-i theta P / 2), adds Im<lambda|P|psi> = 2 Re<lambda|dG/dtheta|psi_prev>.
//
// A state-dependent channel (Algorithm 1's state-dependent branch) is decided
// in the forward preparation as in a batched run, and the state at its decision
// is checkpointed.  With the chosen operator G = K_k / sqrt(p_k) held fixed,
// 2 Re<lambda|dpsi> is d<phi|O|phi> / <phi|phi> for the unnormalised path state
// phi (raw K_k): averaged over paths drawn with their probabilities <phi|phi>
// this is the derivative of sum_paths <phi|O|phi>, the pathwise and the
// score-function term together.  The reverse sweep cannot un-apply a singular
// K_k: at the channel it restores psi from the checkpoint and applies G^dagger
// to lambda alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "host.hpp"
#include "jit.hpp"
#include "kernels.hpp"

namespace ptsbe {

template <typename V>
DenseArgs<V> dense_args(const Plan& P, const ExecStep& ex, V* states, uint8_t* partial, uint8_t* mr_bits,
                        double* mr_norm, uint32_t* status, const double* d_chan_param, uint32_t b0, uint64_t seed,
                        uint32_t cfg, uint64_t alpha0);

namespace {

uint64_t a256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

struct AdjLayout {
  uint64_t status, fwd, adj, aux, routes, psi, lam, partial, ev, scan_part, scan_offs, scan_total, gdot;
  uint64_t mr_partial, mr_bits, mr_norm, rec_info, ckpt, end;
  uint32_t batch, n_tiles, nblk, per_block, per_thread;
  bool share;
};

// The forward preparation shares the error-free prefix as a batched run does
// (plans without state-dependent channels): psi holds two more states, the
// carried one read and written alternately.
bool adjoint_share(const Plan& P, const TrajSet& ts) {
  ptsbe_run_opts o{};
  return prefix_sharing(P, ts, &o);
}

AdjLayout adj_layout(const Plan& P, const TrajSet& ts, uint32_t batch) {
  AdjLayout L{};
  L.share = adjoint_share(P, ts);
  const uint64_t N = 1ull << P.n;
  const uint64_t esz = P.precision == PTSBE_C64 ? 8 : 16;
  const uint64_t B = ts.m.size();
  const uint32_t k_adj = P.adj.passes.empty() ? (uint32_t)P.n : (uint32_t)P.adj.passes[0].k;
  const uint64_t n_dot = P.adj.dot_param.size();
  L.batch = batch;
  // compiled sweeps write one partial per wavefront; room for that either way
  L.n_tiles = (1u << (P.n - k_adj)) * (k_adj >= kMinRegTile ? jit_adjoint_waves(k_adj) : 1u);
  L.per_block = (uint32_t)std::min<uint64_t>(N, kScanBlock);
  L.nblk = (uint32_t)(N / L.per_block);
  L.per_thread = std::max<uint32_t>(1, L.per_block / 256);
  uint64_t o = 0;
  L.status = o; o = a256(o + 16);
  L.fwd = o; o = a256(o + ts.table_blob.size());
  L.adj = o; o = a256(o + ts.adj_blob.size());
  L.aux = o; o = a256(o + B * 8 + std::max<uint64_t>(1, n_dot) * 4);   // weights, dot -> parameter
  const uint64_t n_batches = (B + batch - 1) / std::max<uint32_t>(batch, 1);
  L.routes = o;
  if (L.share) o = a256(o + P.exec.size() * (B + n_batches) * sizeof(uint2));
  L.psi = o; o = a256(o + (uint64_t)(batch + (L.share ? 2 : 0)) * N * esz);
  L.lam = o; o = a256(o + (uint64_t)batch * N * esz);
  L.partial = o; o = a256(o + B * L.n_tiles * std::max<uint64_t>(1, n_dot) * 8);
  L.ev = o; o = a256(o + B * 8);
  L.scan_part = o; o = a256(o + (uint64_t)batch * L.nblk * 8);
  L.scan_offs = o; o = a256(o + (uint64_t)batch * L.nblk * 8);
  L.scan_total = o; o = a256(o + (uint64_t)batch * 8);
  L.gdot = o; o = a256(o + std::max<uint64_t>(1, n_dot) * 8);
  // state-dependent channels: decision partials, record entries, their data,
  // and one checkpointed state per channel step and resident trajectory
  const uint64_t nm = (uint64_t)P.n_measure, ng = (uint64_t)P.n_general;
  L.mr_partial = o; if (nm) o = a256(o + (uint64_t)batch * L.nblk * (kMaxGroup + 1) * 8);
  L.mr_bits = o; if (nm) o = a256(o + B * nm);
  L.mr_norm = o; if (nm) o = a256(o + B * nm * 8);
  L.rec_info = o; if (ng) o = a256(o + nm * 8 + P.rec_info.chan_param.size() * 8);
  L.ckpt = o; o = a256(o + ng * (uint64_t)batch * N * esz);
  L.end = o;
  return L;
}

ptsbe_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return PTSBE_OK;
  return fail(PTSBE_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define CK(expr, what)                           \
  do {                                           \
    ptsbe_status _s = hip_check((expr), (what)); \
    if (_s != PTSBE_OK) return _s;               \
  } while (0)

template <typename V>
PassArgs<V> pass_args(const Plan& P, uint8_t* tb, const TableLayout& T, uint32_t n_passes, V* states) {
  PassArgs<V> pa{};
  pa.passes = reinterpret_cast<const DPass*>(tb + T.passes);
  pa.ops = reinterpret_cast<const DOp*>(tb + T.ops);
  pa.slot_default = reinterpret_cast<const uint32_t*>(tb + T.slot_default);
  pa.pool = reinterpret_cast<const V*>(tb + T.pool);
  pa.ov_off = reinterpret_cast<const uint32_t*>(tb + T.ov_off);
  pa.ov = reinterpret_cast<const DOverride*>(tb + T.ov);
  pa.states = states;
  pa.N = 1ull << P.n;
  pa.n = (uint32_t)P.n;
  pa.n_passes = n_passes;
  pa.n_measure = 0;
  pa.swz = P.swizzle ? 1u : 0u;
  return pa;
}

template <typename V>
ptsbe_status adjoint_typed(const Plan& P, TrajSet& ts, const double* coef, const uint64_t* zmask, uint32_t n_terms,
                           uint64_t seed, uint32_t cfg, uint8_t* ws, const AdjLayout& L, double* d_expval,
                           double* d_grad, hipStream_t s) {
  // every reverse-sweep pass compiled, or none (the partial layouts differ)
  bool compiled = P.use_jit && !P.adj.passes.empty();
  for (uint32_t p = 0; compiled && p < P.adj.passes.size(); ++p) compiled = jit_has_adjoint(P, p);
  const uint32_t B = (uint32_t)ts.m.size();
  const uint64_t N = 1ull << P.n;
  const uint32_t n_dot = (uint32_t)P.adj.dot_param.size();
  CK(hipMemcpyAsync(ws + L.fwd, ts.table_blob.data(), ts.table_blob.size(), hipMemcpyHostToDevice, s), "table upload");
  CK(hipMemcpyAsync(ws + L.adj, ts.adj_blob.data(), ts.adj_blob.size(), hipMemcpyHostToDevice, s), "table upload");
  // weights and the dot -> parameter map live with the plan's host data for the whole call
  std::vector<uint8_t>& aux = ts.adj_aux;
  aux.assign(B * 8 + std::max<uint32_t>(1, n_dot) * 4, 0);
  const std::vector<double> wts = ensemble_weights(ts);
  if (B) std::memcpy(aux.data(), wts.data(), 8 * (size_t)B);
  for (uint32_t d = 0; d < n_dot; ++d) {
    const uint32_t p = (uint32_t)P.adj.dot_param[d];
    std::memcpy(aux.data() + B * 8 + 4 * d, &p, 4);
  }
  CK(hipMemcpyAsync(ws + L.aux, aux.data(), aux.size(), hipMemcpyHostToDevice, s), "weights upload");
  // launch routes of the forward preparation under prefix sharing
  std::vector<uint32_t>& routes = ts.route_host;
  std::vector<uint32_t>& route_off = ts.route_off;
  routes.clear();
  route_off.clear();
  ts.eff_host.clear();
  const uint32_t E = (uint32_t)P.exec.size();
  if (L.share) {
    std::vector<uint32_t> off;
    for (uint32_t b0 = 0; b0 < B; b0 += L.batch) {
      build_routes(P, ts, b0, std::min<uint32_t>(L.batch, B - b0), routes, off, ts.eff_host);
      route_off.insert(route_off.end(), off.begin(), off.end());
    }
    CK(hipMemcpyAsync(ws + L.routes, routes.data(), routes.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s),
       "route upload");
  }
  const uint2* d_routes = reinterpret_cast<const uint2*>(ws + L.routes);
  const uint32_t nm = (uint32_t)P.n_measure;
  const uint32_t* d_rec_chan = nullptr;
  const uint32_t* d_rec_gidx = nullptr;
  const double* d_chan_param = nullptr;
  if (P.n_general) {
    uint8_t* ri = ws + L.rec_info;
    CK(hipMemcpyAsync(ri, P.rec_info.rec_chan.data(), (size_t)nm * 4, hipMemcpyHostToDevice, s), "record upload");
    CK(hipMemcpyAsync(ri + (size_t)nm * 4, P.rec_info.rec_gidx.data(), (size_t)nm * 4, hipMemcpyHostToDevice, s),
       "record upload");
    CK(hipMemcpyAsync(ri + (size_t)nm * 8, P.rec_info.chan_param.data(), P.rec_info.chan_param.size() * 8,
                      hipMemcpyHostToDevice, s),
       "record upload");
    d_rec_chan = reinterpret_cast<const uint32_t*>(ri);
    d_rec_gidx = reinterpret_cast<const uint32_t*>(ri + (size_t)nm * 4);
    d_chan_param = reinterpret_cast<const double*>(ri + (size_t)nm * 8);
  }
  uint32_t* status = reinterpret_cast<uint32_t*>(ws + L.status);
  CK(launch_fill_u32(status, 0, 4, s), "status reset");
  uint8_t* mr_bits = ws + L.mr_bits;
  double* mr_norm = reinterpret_cast<double*>(ws + L.mr_norm);
  V* ckpt = reinterpret_cast<V*>(ws + L.ckpt);
  const uint64_t state_bytes = N * sizeof(V);
  const double* w = reinterpret_cast<const double*>(ws + L.aux);
  const uint32_t* dot_param = reinterpret_cast<const uint32_t*>(ws + L.aux + B * 8);
  V* psi = reinterpret_cast<V*>(ws + L.psi);
  V* lam = reinterpret_cast<V*>(ws + L.lam);
  double* ev = reinterpret_cast<double*>(ws + L.ev);
  double* partial = reinterpret_cast<double*>(ws + L.partial);
  PassArgs<V> fa = pass_args<V>(P, ws + L.fwd, ts.layout, (uint32_t)P.passes.size(), psi);
  fa.mr_bits = mr_bits;
  fa.mr_norm = mr_norm;
  fa.n_measure = nm;
  AdjArgs<V> aa{};
  aa.p = pass_args<V>(P, ws + L.adj, ts.adj_layout, (uint32_t)P.adj.passes.size(), psi);
  aa.lam = lam;
  aa.partial = partial;
  aa.n_dot = n_dot;
  fa.carrier_t = B;
  for (uint32_t b0 = 0, bi = 0; b0 < B; b0 += L.batch, ++bi) {
    const uint32_t bb = std::min<uint32_t>(L.batch, B - b0);
    fa.t0 = b0;
    fa.carrier0 = bb;
    aa.p.t0 = b0;
    for (uint32_t e = 0; e < E; ++e) {
      const ExecStep& ex = P.exec[e];
      if (ex.pass < 0) {
        // one state-dependent channel: checkpoint the state, then decide
        if (ex.mr_index.size() != 1 || !d_rec_chan || P.rec_info.rec_chan[ex.mr_index[0]] == 0xffffffffu)
          return fail(PTSBE_E_UNSUPPORTED, "adjoint: measure-reset steps are not supported");
        const uint32_t g = P.rec_info.rec_gidx[ex.mr_index[0]];
        CK(hipMemcpyAsync(ckpt + ((uint64_t)g * L.batch) * N, psi, (size_t)bb * state_bytes, hipMemcpyDeviceToDevice,
                          s),
           "checkpoint");
        if (ex.dense) {
          CK(launch_dense_channel<V>(dense_args<V>(P, ex, psi, ws + L.mr_partial, mr_bits, mr_norm, status,
                                                   d_chan_param, b0, seed, cfg, ts.alpha0),
                                     bb, s),
             "state-dependent channel");
          continue;
        }
        MarginalArgs<V> ma{};
        ma.swz = fa.swz;
        ma.states = psi;
        ma.partial = reinterpret_cast<double*>(ws + L.mr_partial);
        ma.N = N;
        ma.nblk = L.nblk;
        ma.per_block = L.per_block;
        ma.nq = 1;
        ma.q[0] = (uint32_t)ex.mr_qubits[0];
        MrDecideArgs da{};
        da.partial = ma.partial;
        da.mr_bits = mr_bits;
        da.mr_norm = mr_norm;
        da.status = status;
        da.tol = 1e-6;
        da.nblk = L.nblk;
        da.nq = 1;
        da.t0 = b0;
        da.n_measure = nm;
        da.rec_chan = d_rec_chan;
        da.rec_gidx = d_rec_gidx;
        da.chan_param = d_chan_param;
        da.seed = seed;
        da.cfg = cfg;
        da.alpha0 = ts.alpha0;
        da.carries_norm = 1u;
        da.idx[0] = (uint32_t)ex.mr_index[0];
        CK(launch_marginal<V>(ma, da, bb, s), "state-dependent channel");
        continue;
      }
      const Pass& ps = P.passes[ex.pass];
      fa.pass = (uint32_t)ex.pass;
      uint32_t rows = bb;
      fa.route = nullptr;
      if (L.share) {
        const uint32_t r0 = route_off[(size_t)bi * (E + 1) + e], r1 = route_off[(size_t)bi * (E + 1) + e + 1];
        rows = r1 - r0;
        fa.route = d_routes + r0;
      }
      if (!rows) continue;
      if (jit_has(P, (uint32_t)ex.pass)) {
        CK(jit_launch<V>(P, (uint32_t)ex.pass, fa, rows, s), "compiled forward");
      } else {
        if (ps.k > 12)  // the generic kernels hold at most 12-qubit tiles
          return fail(PTSBE_E_UNSUPPORTED, "forward pass " + std::to_string(ex.pass) +
                                               " has a 13-qubit tile and no compiled kernel");
        CK(launch_pass<V>(fa, (uint32_t)ps.k, (uint32_t)ps.slots.size(), (uint32_t)ps.ops.size(), rows, s),
           "forward");
      }
    }
    ScanArgs<V> sa{};
    sa.swz = fa.swz;
    sa.states = psi;
    sa.partial = reinterpret_cast<double*>(ws + L.scan_part);
    sa.offs = reinterpret_cast<double*>(ws + L.scan_offs);
    sa.N = N;
    sa.nblk = L.nblk;
    sa.per_block = L.per_block;
    sa.per_thread = L.per_thread;
    double* total = reinterpret_cast<double*>(ws + L.scan_total);
    CK(launch_norm<V>(sa, bb, total, s), "norm");
    ExpArgs<V> ea{};
    ea.swz = fa.swz;
    ea.states = psi;
    ea.partial = sa.partial;
    ea.N = N;
    ea.nblk = L.nblk;
    ea.per_block = L.per_block;
    ea.n_terms = n_terms;
    ObsArgs<V> oa{};
    oa.swz = fa.swz;
    oa.psi = psi;
    oa.lam = lam;
    oa.N = N;
    oa.n_terms = n_terms;
    for (uint32_t j = 0; j < n_terms; ++j) {
      ea.coef[j] = oa.coef[j] = coef[j];
      ea.zmask[j] = oa.zmask[j] = zmask[j];
    }
    CK(launch_expval<V>(ea, total, ev, bb, b0, s), "expectation");
    CK(launch_obs_apply<V>(oa, bb, s), "lambda");
    for (const ExecStep& ex : P.adj.exec) {
      if (ex.pass < 0) {
        // state-dependent channel: psi from its checkpoint, lambda <- G^dagger lambda
        const uint32_t r = (uint32_t)ex.mr_index[0];
        CK(hipMemcpyAsync(psi, ckpt + ((uint64_t)ex.restore * L.batch) * N, (size_t)bb * state_bytes,
                          hipMemcpyDeviceToDevice, s),
           "checkpoint restore");
        if (ex.dense) {
          DenseArgs<V> da = dense_args<V>(P, ex, psi, ws + L.mr_partial, mr_bits, mr_norm, status, d_chan_param, b0,
                                          seed, cfg, ts.alpha0);
          da.lam = lam;
          CK(launch_dense_lam_adjoint<V>(da, bb, s), "state-dependent channel adjoint");
          continue;
        }
        GchAdjArgs<V> ga{};
        ga.swz = fa.swz;
        ga.lam = lam;
        ga.mr_bits = mr_bits;
        ga.mr_norm = mr_norm;
        ga.chan = d_chan_param + P.rec_info.rec_chan[r];
        ga.N = N;
        ga.q = (uint32_t)ex.mr_qubits[0];
        ga.rec = r;
        ga.n_measure = nm;
        ga.t0 = b0;
        CK(launch_gch_lam_adjoint<V>(ga, bb, s), "state-dependent channel adjoint");
        continue;
      }
      const Pass& ps = P.adj.passes[ex.pass];
      aa.p.pass = (uint32_t)ex.pass;
      if (compiled)
        CK(jit_adjoint_launch<V>(P, (uint32_t)ex.pass, aa, bb, s), "compiled reverse sweep");
      else
        CK(launch_adjoint_pass<V>(aa, (uint32_t)ps.k, (uint32_t)ps.slots.size(), bb, s), "reverse sweep");
    }
  }
  const uint32_t k_adj = P.adj.passes.empty() ? (uint32_t)P.n : (uint32_t)P.adj.passes[0].k;
  const uint32_t tiles_eff = compiled ? L.n_tiles : (1u << (P.n - k_adj));
  CK(launch_grad_reduce(partial, w, B, tiles_eff, n_dot, reinterpret_cast<double*>(ws + L.gdot), dot_param,
                        (uint32_t)P.n_params, d_grad, ev, d_expval, s),
     "gradient reduction");
  return PTSBE_OK;
}

ptsbe_status check_adjoint(const Plan& P, const TrajSet& ts, const double* params, const double* coef,
                           const uint64_t* zmask, uint32_t n_terms) {
  if (!P.has_adjoint)
    return fail(PTSBE_E_UNSUPPORTED,
                "adjoint gradient needs parametrised gates and no measure-reset / projection operations");
  if (!params) return fail(PTSBE_E_ARG, "params required");
  if (n_terms == 0 || n_terms > 64 || !coef || !zmask)
    return fail(PTSBE_E_ARG, "observable: 1..64 Z-string terms with coefficients and masks");
  if (P.n < 64)
    for (uint32_t j = 0; j < n_terms; ++j)
      if (zmask[j] >> P.n) return fail(PTSBE_E_ARG, "observable names a qubit >= n");
  if (ts.m.empty()) return fail(PTSBE_E_ARG, "empty trajectory set");
  return PTSBE_OK;
}

}  // namespace

ptsbe_status adjoint_workspace_size(const Plan& P, TrajSet& ts, const double* params, uint32_t max_batch,
                                    size_t* bytes) {
  if (!P.has_adjoint)
    return fail(PTSBE_E_UNSUPPORTED,
                "adjoint gradient needs parametrised gates and no measure-reset / projection operations");
  if (!params) return fail(PTSBE_E_ARG, "params required");
  if (ts.m.empty()) return fail(PTSBE_E_ARG, "empty trajectory set");
  std::lock_guard<std::mutex> lk(ts.mu);
  ptsbe_status st = build_tables(ts, params, 4096);
  if (st != PTSBE_OK) return st;
  st = build_adj_tables(ts, params);
  if (st != PTSBE_OK) return st;
  uint32_t batch = std::min<uint32_t>((uint32_t)ts.m.size(), 65535);
  if (max_batch) batch = std::min(batch, max_batch);
  *bytes = adj_layout(P, ts, batch).end;
  return PTSBE_OK;
}

ptsbe_status adjoint_grad(const Plan& P, TrajSet& ts, const double* params, const double* coef,
                          const uint64_t* zmask, uint32_t n_terms, uint64_t seed, uint32_t cfg, void* d_ws,
                          size_t ws_bytes, double* d_expval, double* d_grad, void* stream) {
  ptsbe_status st = check_adjoint(P, ts, params, coef, zmask, n_terms);
  if (st != PTSBE_OK) return st;
  if (!d_ws || !d_expval || !d_grad) return fail(PTSBE_E_ARG, "null device pointer");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256) return fail(PTSBE_E_ARG, "workspace must be 256-byte aligned");
  if (P.use_jit) {
    st = jit_build(P);
    if (st != PTSBE_OK) return st;
  }
  std::lock_guard<std::mutex> lk(ts.mu);
  st = build_tables(ts, params, 4096);
  if (st != PTSBE_OK) return st;
  st = build_adj_tables(ts, params);
  if (st != PTSBE_OK) return st;
  const uint32_t B = (uint32_t)ts.m.size();
  uint32_t batch = std::min<uint32_t>(B, 65535);
  AdjLayout L = adj_layout(P, ts, batch);
  while (L.end > ws_bytes && batch > 1) {
    batch = std::max<uint32_t>(1, batch / 2);
    L = adj_layout(P, ts, batch);
  }
  if (L.end > ws_bytes)
    return fail(PTSBE_E_OOM, "workspace of " + std::to_string(ws_bytes) + " bytes is below the " +
                                 std::to_string(L.end) + " bytes needed");
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (P.precision == PTSBE_C64)
    return adjoint_typed<float2>(P, ts, coef, zmask, n_terms, seed, cfg, ws, L, d_expval, d_grad, s);
  return adjoint_typed<double2>(P, ts, coef, zmask, n_terms, seed, cfg, ws, L, d_expval, d_grad, s);
}

}  // namespace ptsbe
