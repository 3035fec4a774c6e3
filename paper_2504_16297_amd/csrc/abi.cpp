// extern "C" entry points of libptsbe: argument checks and exception fences
// around the planner, the PTS samplers and the batched executor.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "host.hpp"
#include "jit.hpp"

namespace ptsbe {
const char* last_error_cstr();
ptsbe_status sample_kraus(const std::shared_ptr<Plan>& plan, const ptsbe_pts_opts* o, ptsbe_trajset_t* out);
ptsbe_status trajset_from_records(const std::shared_ptr<Plan>& plan, uint32_t n, const uint32_t* off,
                                  const uint32_t* site, const uint8_t* kraus, const uint64_t* m, uint64_t alpha0,
                                  ptsbe_trajset_t* out);
ptsbe_status trajset_slice(const TrajSet& ts, uint32_t b, uint32_t e, ptsbe_trajset_t* out);
ptsbe_status workspace_size(const Plan& P, TrajSet& ts, const ptsbe_run_opts* o, size_t* bytes);
ptsbe_status run_batch(const Plan& P, TrajSet& ts, const ptsbe_run_opts* o, void* d_ws, size_t ws_bytes,
                       void* d_bits, uint32_t* d_traj, uint64_t capacity, uint8_t* d_mr_bits, void* stream,
                       hipGraphExec_t* graph_out = nullptr, bool no_alloc = false,
                       uint32_t* d_status = nullptr);
ptsbe_status run_status(const void* d_ws, void* stream);
ptsbe_status adjoint_grad(const Plan& P, TrajSet& ts, const double* params, const double* coef,
                          const uint64_t* zmask, uint32_t n_terms, uint64_t seed, uint32_t cfg, void* d_ws,
                          size_t ws_bytes, double* d_expval, double* d_grad, void* stream);
ptsbe_status adjoint_workspace_size(const Plan& P, TrajSet& ts, const double* params, uint32_t max_batch,
                                    size_t* bytes);
}  // namespace ptsbe

using namespace ptsbe;

#define FENCE(...)                                                   \
  try {                                                              \
    __VA_ARGS__                                                      \
  } catch (const std::bad_alloc&) {                                  \
    return fail(PTSBE_E_OOM, "host allocation failed");              \
  } catch (const std::exception& e) {                                \
    return fail(PTSBE_E_ARG, std::string("internal error: ") + e.what()); \
  } catch (...) {                                                    \
    return fail(PTSBE_E_ARG, "internal error");                      \
  }

extern "C" {

const char* ptsbe_last_error(void) { return last_error_cstr(); }

const char* ptsbe_version(void) { return "ptsbe-gfx950 0.1.0"; }

ptsbe_status ptsbe_plan(const ptsbe_circuit* circuit, const ptsbe_noise_model* noise, const ptsbe_plan_opts* opts,
                        ptsbe_plan_t* out) {
  FENCE({
    if (!out) return fail(PTSBE_E_ARG, "null output handle");
    *out = nullptr;
    std::shared_ptr<Plan> p;
    ptsbe_status st = build_plan(circuit, noise, opts, &p);
    if (st != PTSBE_OK) return st;
    auto* h = new ptsbe_plan_s;
    h->plan = p;
    *out = h;
    return PTSBE_OK;
  })
}

ptsbe_status ptsbe_plan_compile(ptsbe_plan_t plan, uint32_t* n_kernels, double* seconds) {
  FENCE({
    if (!plan) return fail(PTSBE_E_ARG, "null plan");
    const Plan& P = *plan->plan;
    ptsbe_status st = jit_build(P);
    if (n_kernels) *n_kernels = (uint32_t)P.jit->names.size();
    if (seconds) *seconds = P.jit->compile_seconds;
    return st;
  })
}

ptsbe_status ptsbe_plan_pass_source(ptsbe_plan_t plan, uint32_t pass, uint32_t adjoint, char* out, size_t* len) {
  FENCE({
    if (!plan || !len) return fail(PTSBE_E_ARG, "null argument");
    const Plan& P = *plan->plan;
    const std::vector<Pass>& passes = adjoint ? P.adj.passes : P.passes;
    if (pass >= passes.size()) return fail(PTSBE_E_ARG, "pass index out of range");
    const std::string src =
        jit_pass_source(passes[pass], P.n, P.precision, "ptsbe_pass", P.half_tile_lds, nullptr, adjoint != 0,
                        P.waves, P.swizzle, P.nontemporal, P.tiles_per_block);
    if (out) {
      if (*len < src.size() + 1) return fail(PTSBE_E_ARG, "output buffer too small");
      std::memcpy(out, src.c_str(), src.size() + 1);
    }
    *len = src.size() + 1;
    return PTSBE_OK;
  })
}

ptsbe_status ptsbe_plan_get_info(ptsbe_plan_t plan, ptsbe_plan_info* out) {
  if (!plan || !out) return fail(PTSBE_E_ARG, "null argument");
  const Plan& P = *plan->plan;
  std::memset(out, 0, sizeof(*out));
  out->n_qubits = (uint32_t)P.n;
  out->n_sites = (uint32_t)P.sites.size();
  out->n_params = (uint32_t)P.n_params;
  out->n_measure = (uint32_t)P.n_measure;
  out->n_passes = (uint32_t)P.passes.size();
  out->n_steps = (uint32_t)P.exec.size();
  out->precision = (uint32_t)P.precision;
  out->tile_qubits = (uint32_t)std::min(P.n, P.tile_bits);
  uint32_t mk = 0;
  for (auto& c : P.channels) mk = std::max<uint32_t>(mk, (uint32_t)c.K);
  out->max_kraus = mk;
  out->total_kraus = (uint32_t)P.site_p.size();
  out->swizzled = P.swizzle ? 1u : 0u;
  return PTSBE_OK;
}

ptsbe_status ptsbe_plan_get_sites(ptsbe_plan_t plan, uint32_t* offsets, double* probs, uint32_t* qubits) {
  if (!plan) return fail(PTSBE_E_ARG, "null plan");
  const Plan& P = *plan->plan;
  if (offsets) std::memcpy(offsets, P.site_off.data(), P.site_off.size() * 4);
  if (probs && !P.site_p.empty()) std::memcpy(probs, P.site_p.data(), P.site_p.size() * 8);
  if (qubits)
    for (size_t s = 0; s < P.sites.size(); ++s) {
      qubits[2 * s] = (uint32_t)P.sites[s].q[0];
      qubits[2 * s + 1] = P.sites[s].nq > 1 ? (uint32_t)P.sites[s].q[1] : 0xffffffffu;
    }
  return PTSBE_OK;
}

ptsbe_status ptsbe_plan_get_site_ops(ptsbe_plan_t plan, uint32_t* op_index, uint32_t* tag, uint32_t* origin) {
  if (!plan) return fail(PTSBE_E_ARG, "null plan");
  const Plan& P = *plan->plan;
  for (size_t s = 0; s < P.sites.size(); ++s) {
    if (op_index) op_index[s] = P.sites[s].op;
    if (tag) tag[s] = P.sites[s].tag;
    if (origin) origin[s] = P.sites[s].origin;
  }
  return PTSBE_OK;
}

ptsbe_status ptsbe_plan_get_record_info(ptsbe_plan_t plan, uint32_t* channel, uint32_t* gidx) {
  if (!plan) return fail(PTSBE_E_ARG, "null plan");
  const Plan& P = *plan->plan;
  std::vector<uint32_t> ch(P.n_measure, 0xffffffffu), gi(P.n_measure, 0u);
  for (const Step& st : P.steps)
    if (st.kind == ST_GCH) {
      ch[st.mr] = (uint32_t)st.chan;
      gi[st.mr] = (uint32_t)st.gidx;
    }
  if (channel) std::copy(ch.begin(), ch.end(), channel);
  if (gidx) std::copy(gi.begin(), gi.end(), gidx);
  return PTSBE_OK;
}

void ptsbe_plan_destroy(ptsbe_plan_t plan) { delete plan; }

ptsbe_status ptsbe_sample_kraus(ptsbe_plan_t plan, const ptsbe_pts_opts* opts, ptsbe_trajset_t* out) {
  FENCE({
    if (!plan || !opts || !out) return fail(PTSBE_E_ARG, "null argument");
    *out = nullptr;
    return sample_kraus(plan->plan, opts, out);
  })
}

ptsbe_status ptsbe_trajset_from_records(ptsbe_plan_t plan, uint32_t n_traj, const uint32_t* rec_off,
                                        const uint32_t* rec_site, const uint8_t* rec_kraus, const uint64_t* m,
                                        uint64_t alpha0, ptsbe_trajset_t* out) {
  FENCE({
    if (!plan || !out) return fail(PTSBE_E_ARG, "null argument");
    *out = nullptr;
    return trajset_from_records(plan->plan, n_traj, rec_off, rec_site, rec_kraus, m, alpha0, out);
  })
}

ptsbe_status ptsbe_trajset_slice(ptsbe_trajset_t ts, uint32_t begin, uint32_t end, ptsbe_trajset_t* out) {
  FENCE({
    if (!ts || !out) return fail(PTSBE_E_ARG, "null argument");
    *out = nullptr;
    return trajset_slice(*ts->ts, begin, end, out);
  })
}

ptsbe_status ptsbe_trajset_get(ptsbe_trajset_t h, uint32_t* n_traj, uint64_t* total_shots, uint32_t* n_entries,
                               uint64_t* alpha0, uint64_t* m, double* p, uint64_t* count, uint32_t* rec_off,
                               uint32_t* rec_site, uint8_t* rec_kraus) {
  if (!h) return fail(PTSBE_E_ARG, "null trajectory set");
  const TrajSet& ts = *h->ts;
  size_t B = ts.m.size();
  if (n_traj) *n_traj = (uint32_t)B;
  if (total_shots) *total_shots = ts.total_shots;
  if (n_entries) *n_entries = (uint32_t)ts.rec_site.size();
  if (alpha0) *alpha0 = ts.alpha0;
  // copies skip empty arrays (an empty vector's data() may be null)
  auto out = [](void* dst, const void* src, size_t bytes) {
    if (dst && bytes) std::memcpy(dst, src, bytes);
  };
  out(m, ts.m.data(), B * 8);
  out(p, ts.p.data(), B * 8);
  out(count, ts.count.data(), B * 8);
  out(rec_off, ts.rec_off.data(), (B + 1) * 4);
  out(rec_site, ts.rec_site.data(), ts.rec_site.size() * 4);
  out(rec_kraus, ts.rec_kraus.data(), ts.rec_kraus.size());
  return PTSBE_OK;
}

ptsbe_status ptsbe_site_selection(ptsbe_plan_t plan, const ptsbe_site_filter* f, uint8_t* flags) {
  FENCE({
    if (!plan || !f || !flags) return fail(PTSBE_E_ARG, "null argument");
    const Plan& P = *plan->plan;
    auto in = [](const uint32_t* v, uint32_t n, uint32_t x) {
      if (!v) return true;
      for (uint32_t i = 0; i < n; ++i)
        if (v[i] == x) return true;
      return false;
    };
    for (size_t s = 0; s < P.sites.size(); ++s) {
      const Site& st = P.sites[s];
      bool ok = in(f->tags, f->n_tags, st.tag) && in(f->ops, f->n_ops, st.op) &&
                in(f->origins, f->n_origins, st.origin);
      for (int j = 0; j < st.nq && ok; ++j) ok = in(f->qubits, f->n_qubits, (uint32_t)st.q[j]);
      const uint32_t b = P.site_off[s], e = P.site_off[s + 1];
      flags[b] = 1;
      for (uint32_t k = 1; k < e - b; ++k) flags[b + k] = (ok && in(f->kraus, f->n_kraus, k)) ? 1 : 0;
    }
    return PTSBE_OK;
  })
}

ptsbe_status ptsbe_trajset_weights(ptsbe_trajset_t h, double* w) {
  FENCE({
    if (!h || !w) return fail(PTSBE_E_ARG, "null argument");
    const std::vector<double> v = ensemble_weights(*h->ts);
    std::copy(v.begin(), v.end(), w);
    return PTSBE_OK;
  })
}

void ptsbe_trajset_destroy(ptsbe_trajset_t ts) { delete ts; }

ptsbe_status ptsbe_workspace_size(ptsbe_plan_t plan, ptsbe_trajset_t ts, const ptsbe_run_opts* opts, size_t* bytes) {
  FENCE({
    if (!plan || !ts || !bytes) return fail(PTSBE_E_ARG, "null argument");
    if (ts->ts->plan.get() != plan->plan.get()) return fail(PTSBE_E_ARG, "trajectory set belongs to another plan");
    if (opts && opts->mode == PTSBE_RUN_ADJOINT)
      return adjoint_workspace_size(*plan->plan, *ts->ts, opts->params, opts->max_batch, bytes);
    return workspace_size(*plan->plan, *ts->ts, opts, bytes);
  })
}

ptsbe_status ptsbe_run_batch(ptsbe_plan_t plan, ptsbe_trajset_t ts, const ptsbe_run_opts* opts, void* d_ws,
                             size_t ws_bytes, void* d_bits, uint32_t* d_traj, uint64_t capacity, uint8_t* d_mr_bits,
                             void* stream) {
  FENCE({
    if (!plan || !ts) return fail(PTSBE_E_ARG, "null argument");
    if (ts->ts->plan.get() != plan->plan.get()) return fail(PTSBE_E_ARG, "trajectory set belongs to another plan");
    return run_batch(*plan->plan, *ts->ts, opts, d_ws, ws_bytes, d_bits, d_traj, capacity, d_mr_bits, stream);
  })
}

ptsbe_status ptsbe_graph_create(ptsbe_plan_t plan, ptsbe_trajset_t ts, const ptsbe_run_opts* opts, void* d_ws,
                                size_t ws_bytes, void* d_bits, uint32_t* d_traj, uint64_t capacity,
                                uint8_t* d_mr_bits, void* stream, ptsbe_graph_t* out) {
  FENCE({
    if (!plan || !ts || !out) return fail(PTSBE_E_ARG, "null argument");
    if (ts->ts->plan.get() != plan->plan.get()) return fail(PTSBE_E_ARG, "trajectory set belongs to another plan");
    hipGraphExec_t exec = nullptr;
    ptsbe_status st =
        run_batch(*plan->plan, *ts->ts, opts, d_ws, ws_bytes, d_bits, d_traj, capacity, d_mr_bits, stream, &exec);
    if (st != PTSBE_OK) return st;
    ptsbe_graph_s* g = new ptsbe_graph_s;
    g->plan = plan->plan;
    g->ts = ts->ts;
    g->exec = exec;
    *out = g;
    return PTSBE_OK;
  })
}

ptsbe_status ptsbe_graph_launch(ptsbe_graph_t g, void* stream) {
  if (!g || !g->exec) return fail(PTSBE_E_ARG, "null graph");
  hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(PTSBE_E_DEVICE, std::string("graph launch: ") + hipGetErrorString(e));
  return PTSBE_OK;
}

void ptsbe_graph_destroy(ptsbe_graph_t g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  delete g;
}

ptsbe_status ptsbe_trajset_tables(ptsbe_trajset_t h, const double* params, uint32_t sort_chunk, void* out,
                                  size_t* bytes, uint64_t* offsets) {
  FENCE({
    if (!h || !bytes) return fail(PTSBE_E_ARG, "null argument");
    TrajSet& ts = *h->ts;
    uint32_t chunk = sort_chunk ? sort_chunk : 4096;
    if (chunk < 256 || chunk > 4096 || (chunk & (chunk - 1)))
      return fail(PTSBE_E_ARG, "sort_chunk must be a power of two in 256..4096");
    if (ts.plan->n_params && !params) return fail(PTSBE_E_ARG, "the circuit has parameters: params required");
    std::lock_guard<std::mutex> lk(ts.mu);
    ptsbe_status st = build_tables(ts, params, chunk);
    if (st != PTSBE_OK) return st;
    if (out) {
      if (*bytes < ts.table_blob.size()) return fail(PTSBE_E_ARG, "output buffer too small");
      std::memcpy(out, ts.table_blob.data(), ts.table_blob.size());
    }
    *bytes = ts.table_blob.size();
    if (offsets) {
      const TableLayout& L = ts.layout;
      const uint64_t v[16] = {L.passes, L.ops,    L.slot_default, L.pool,  L.ov_off,  L.ov,
                              L.shot_off, L.chunk_off, L.exec,    L.n_passes, L.n_ops, L.n_slots,
                              L.n_pool, L.n_ov,   L.n_exec,       L.total};
      std::memcpy(offsets, v, sizeof(v));
    }
    return PTSBE_OK;
  })
}

ptsbe_status ptsbe_trajset_adjoint_tables(ptsbe_trajset_t h, const double* params, void* out, size_t* bytes,
                                          uint64_t* offsets, uint32_t* n_dot, uint32_t* dot_param) {
  FENCE({
    if (!h || !bytes) return fail(PTSBE_E_ARG, "null argument");
    TrajSet& ts = *h->ts;
    const Plan& P = *ts.plan;
    if (!params) return fail(PTSBE_E_ARG, "params required");
    std::lock_guard<std::mutex> lk(ts.mu);
    ptsbe_status st = build_adj_tables(ts, params);
    if (st != PTSBE_OK) return st;
    if (out) {
      if (*bytes < ts.adj_blob.size()) return fail(PTSBE_E_ARG, "output buffer too small");
      std::memcpy(out, ts.adj_blob.data(), ts.adj_blob.size());
    }
    *bytes = ts.adj_blob.size();
    if (offsets) {
      const TableLayout& L = ts.adj_layout;
      const uint64_t v[16] = {L.passes, L.ops,    L.slot_default, L.pool,  L.ov_off,  L.ov,
                              L.shot_off, L.chunk_off, L.exec,    L.n_passes, L.n_ops, L.n_slots,
                              L.n_pool, L.n_ov,   L.n_exec,       L.total};
      std::memcpy(offsets, v, sizeof(v));
    }
    if (n_dot) *n_dot = (uint32_t)P.adj.dot_param.size();
    if (dot_param)
      for (size_t d = 0; d < P.adj.dot_param.size(); ++d) dot_param[d] = (uint32_t)P.adj.dot_param[d];
    return PTSBE_OK;
  })
}

ptsbe_status ptsbe_run_status(ptsbe_plan_t plan, const void* d_ws, void* stream) {
  FENCE({
    if (!plan) return fail(PTSBE_E_ARG, "null plan");
    return run_status(d_ws, stream);
  })
}

ptsbe_status ptsbe_unique_workspace_size(ptsbe_trajset_t ts, uint32_t max_batch, size_t* bytes) {
  FENCE({
    if (!ts || !bytes) return fail(PTSBE_E_ARG, "null argument");
    return unique_workspace_size(*ts->ts, max_batch, bytes);
  })
}

ptsbe_status ptsbe_unique_shots(ptsbe_trajset_t ts, const void* d_bits, void* d_ws, size_t ws_bytes,
                                uint64_t* d_unique, void* d_pair_index, uint32_t* d_pair_count, void* stream) {
  FENCE({
    if (!ts) return fail(PTSBE_E_ARG, "null trajectory set");
    std::lock_guard<std::mutex> lk(ts->ts->mu);
    return unique_shots(*ts->ts, d_bits, d_ws, ws_bytes, d_unique, d_pair_index, d_pair_count,
                        reinterpret_cast<hipStream_t>(stream));
  })
}

ptsbe_status ptsbe_adjoint_grad(ptsbe_plan_t plan, ptsbe_trajset_t ts, const double* params, const double* obs_coef,
                                const uint64_t* obs_zmask, uint32_t n_terms, uint64_t seed, uint32_t cfg,
                                void* d_ws, size_t ws_bytes, double* d_expval, double* d_grad, void* stream) {
  FENCE({
    if (!plan || !ts) return fail(PTSBE_E_ARG, "null argument");
    if (ts->ts->plan.get() != plan->plan.get()) return fail(PTSBE_E_ARG, "trajectory set belongs to another plan");
    return adjoint_grad(*plan->plan, *ts->ts, params, obs_coef, obs_zmask, n_terms, seed, cfg, d_ws, ws_bytes,
                        d_expval, d_grad, stream);
  })
}

// --------------------------------------------------------------- gate library

static void put(double* out, const Mat& m) {
  for (size_t i = 0; i < m.size(); ++i) {
    out[2 * i] = m[i].real();
    out[2 * i + 1] = m[i].imag();
  }
}

ptsbe_status ptsbe_std_gate(const char* name, const double* params, double* out, uint32_t* nq) {
  if (!name || !out || !nq) return fail(PTSBE_E_ARG, "null argument");
  std::string n(name);
  const double r2 = 1.0 / std::sqrt(2.0);
  Mat m;
  uint32_t q = 1;
  auto need = [&](int k) { return params != nullptr || k == 0; };
  if (n == "U3") {
    if (!need(3)) return fail(PTSBE_E_ARG, "U3 needs 3 parameters");
    double c = std::cos(params[0] / 2), s = std::sin(params[0] / 2);
    m = {cd(c, 0), -std::polar(1.0, params[2]) * s, std::polar(1.0, params[1]) * s,
         std::polar(1.0, params[1] + params[2]) * c};
  } else if (n == "RX" || n == "RY" || n == "RZ") {
    if (!need(1)) return fail(PTSBE_E_ARG, "rotations need 1 parameter");
    m = rot_matrix(n == "RX" ? PTSBE_GEN_X : n == "RY" ? PTSBE_GEN_Y : PTSBE_GEN_Z, params[0]);
  } else if (n == "H") {
    m = {cd(r2, 0), cd(r2, 0), cd(r2, 0), cd(-r2, 0)};
  } else if (n == "X") {
    m = {0, 1, 1, 0};
  } else if (n == "Y") {
    m = {0, cd(0, -1), cd(0, 1), 0};
  } else if (n == "Z") {
    m = {1, 0, 0, -1};
  } else if (n == "S") {
    m = {1, 0, 0, cd(0, 1)};
  } else if (n == "T") {
    m = {1, 0, 0, std::polar(1.0, std::atan(1.0))};
  } else if (n == "CZ") {
    q = 2;
    m = mat_identity(4);
    m[15] = -1;
  } else if (n == "CNOT") {
    // qubits (control, target): index = c + 2 t
    q = 2;
    m.assign(16, 0);
    for (int c = 0; c < 2; ++c)
      for (int t = 0; t < 2; ++t) m[(c + 2 * (t ^ c)) * 4 + c + 2 * t] = 1;
  } else if (n == "SWAP") {
    q = 2;
    m.assign(16, 0);
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) m[(b + 2 * a) * 4 + a + 2 * b] = 1;
  } else {
    return fail(PTSBE_E_ARG, "unknown gate " + n);
  }
  put(out, m);
  *nq = q;
  return PTSBE_OK;
}

ptsbe_status ptsbe_pauli_twirl(uint32_t nq, const double* kraus, uint32_t n_kraus, double* probs) {
  FENCE({ return pauli_twirl_channel(nq, kraus, n_kraus, probs); })
}

ptsbe_status ptsbe_std_channel(const char* name, uint32_t nq, const double* params, double* out, uint32_t* n_kraus) {
  if (!name || !out || !n_kraus || !params) return fail(PTSBE_E_ARG, "null argument");
  std::string n(name);
  const Mat I = mat_identity(2);
  const Mat X = {0, 1, 1, 0}, Y = {0, cd(0, -1), cd(0, 1), 0}, Z = {1, 0, 0, -1};
  const Mat* P[4] = {&I, &X, &Y, &Z};
  auto scaled = [](const Mat& a, double s) {
    Mat r = a;
    for (auto& x : r) x *= s;
    return r;
  };
  auto kron = [](const Mat& a, const Mat& b) {  // a on matrix bit 1, b on bit 0
    Mat r(16);
    for (int r1 = 0; r1 < 2; ++r1)
      for (int c1 = 0; c1 < 2; ++c1)
        for (int r0 = 0; r0 < 2; ++r0)
          for (int c0 = 0; c0 < 2; ++c0) r[(2 * r1 + r0) * 4 + 2 * c1 + c0] = a[r1 * 2 + c1] * b[r0 * 2 + c0];
    return r;
  };
  std::vector<Mat> ks;
  if (n == "depolarizing") {
    double p = params[0];
    if (!(p >= 0 && p <= 1)) return fail(PTSBE_E_ARG, "p must be in [0, 1]");
    if (nq == 1) {
      ks.push_back(scaled(I, std::sqrt(1.0 - p)));
      for (int i = 1; i < 4; ++i) ks.push_back(scaled(*P[i], std::sqrt(p / 3.0)));
    } else if (nq == 2) {
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
          ks.push_back(scaled(kron(*P[a], *P[b]), (a == 0 && b == 0) ? std::sqrt(1.0 - p) : std::sqrt(p / 15.0)));
    } else {
      return fail(PTSBE_E_ARG, "depolarizing acts on 1 or 2 qubits");
    }
  } else if (n == "xflip") {
    double p = params[0];
    ks = {scaled(I, std::sqrt(1.0 - p)), scaled(X, std::sqrt(p))};
  } else if (n == "pauli") {
    double px = params[0], py = params[1], pz = params[2];
    ks = {scaled(I, std::sqrt(1.0 - px - py - pz)), scaled(X, std::sqrt(px)), scaled(Y, std::sqrt(py)),
          scaled(Z, std::sqrt(pz))};
  } else if (n == "u3_mixture") {
    double p = params[0];
    double gg[8];
    uint32_t q1;
    ptsbe_std_gate("U3", params + 1, gg, &q1);
    Mat U = {cd(gg[0], gg[1]), cd(gg[2], gg[3]), cd(gg[4], gg[5]), cd(gg[6], gg[7])};
    ks = {scaled(I, std::sqrt(1.0 - p)), scaled(U, std::sqrt(p))};
  } else if (n == "amplitude_damping") {
    double g = params[0];
    ks = {Mat{1, 0, 0, std::sqrt(1.0 - g)}, Mat{0, std::sqrt(g), 0, 0}};
  } else {
    return fail(PTSBE_E_ARG, "unknown channel " + n);
  }
  size_t d2 = ks[0].size();
  for (size_t k = 0; k < ks.size(); ++k) put(out + 2 * k * d2, ks[k]);
  *n_kraus = (uint32_t)ks.size();
  return PTSBE_OK;
}

}  // extern "C"
