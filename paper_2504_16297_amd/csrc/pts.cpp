// Pre-trajectory sampling (Sec. 3.1) and trajectory sets, plus the per-run
// device tables derived from a trajectory set.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <unordered_map>

#include "host.hpp"
#include "philox.hpp"

namespace ptsbe {

namespace {

// Smallest k with u < p_0 + ... + p_k (prefix sums in order), clamped to the last index.
int categorical(double u, const double* p, int K) {
  double c = 0.0;
  for (int k = 0; k < K; ++k) {
    c += p[k];
    if (u < c) return k;
  }
  return K - 1;
}

using Record = std::vector<std::pair<uint32_t, uint8_t>>;

struct RecordHash {
  size_t operator()(const Record& r) const {
    uint64_t h = 1469598103934665603ull;
    for (auto& e : r) {
      h ^= (uint64_t)e.first * 31 + e.second;
      h *= 1099511628211ull;
    }
    return (size_t)h;
  }
};

double joint_prob(const Plan& P, const Record& rec) {
  double p = 1.0;
  size_t j = 0;
  for (size_t s = 0; s < P.sites.size(); ++s) {
    int k = 0;
    if (j < rec.size() && rec[j].first == s) k = rec[j++].second;
    p *= P.site_p[P.site_off[s] + k];
  }
  return p;
}

std::vector<uint64_t> alloc_multiplicity(const std::vector<uint64_t>& counts, uint64_t T, uint64_t S) {
  size_t B = counts.size();
  std::vector<uint64_t> base(B), rem(B);
  uint64_t sum = 0;
  for (size_t a = 0; a < B; ++a) {
    unsigned __int128 x = (unsigned __int128)counts[a] * S;
    base[a] = (uint64_t)(x / T);
    rem[a] = (uint64_t)(x % T);
    sum += base[a];
  }
  uint64_t left = S - sum;
  std::vector<size_t> order(B);
  for (size_t a = 0; a < B; ++a) order[a] = a;
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return rem[x] > rem[y]; });
  for (uint64_t i = 0; i < left && i < B; ++i) base[order[i]] += 1;
  return base;
}

std::vector<uint64_t> alloc_reweight(const std::vector<double>& p, uint64_t S) {
  size_t B = p.size();
  double P = 0.0;
  for (double v : p) P += v;
  std::vector<uint64_t> base(B);
  std::vector<double> frac(B);
  uint64_t sum = 0;
  for (size_t a = 0; a < B; ++a) {
    double x = (p[a] / P) * (double)S;
    double f = std::floor(x);
    base[a] = (uint64_t)f;
    frac[a] = x - f;
    sum += base[a];
  }
  uint64_t left = S > sum ? S - sum : 0;
  std::vector<size_t> order(B);
  for (size_t a = 0; a < B; ++a) order[a] = a;
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return frac[x] > frac[y]; });
  for (uint64_t i = 0; i < left && i < B; ++i) base[order[i]] += 1;
  return base;
}

struct Item {
  double c;
  uint32_t s;
  uint8_t k;
};

// Selection criteria of a PTS run (operator flags and record-level filters).
struct Criteria {
  const uint8_t* allow = nullptr;  // per (site, k) flags, k >= 1 consulted
  uint32_t min_errors = 0, max_errors = 0, parity = PTSBE_PARITY_ANY;
  const Plan* P = nullptr;
  bool allowed(size_t s, int k) const { return !allow || k == 0 || allow[P->site_off[s] + k]; }
  bool keep(size_t n_err) const {
    if (n_err < min_errors) return false;
    if (max_errors && n_err > max_errors) return false;
    if (parity == PTSBE_PARITY_EVEN && (n_err & 1)) return false;
    if (parity == PTSBE_PARITY_ODD && !(n_err & 1)) return false;
    return true;
  }
  bool any_filter() const { return min_errors || max_errors || parity != PTSBE_PARITY_ANY; }
};

// Most-likely-first selection: records ranked by ascending score
// sum_{(s,k)} -ln(p_{s,k}/p_{s,0}) (summed in ascending (c, s, k) order), ties by
// the record's (s, k) list.  A depth-first walk over the items sorted by cost
// finds every record with score <= tau; tau is bisected until at least k_max
// records qualify, then the qualifying records are sorted and cut.
// Selection criteria restrict the items to allowed operators; only records the
// record-level filters keep are counted (and collected), and no record grows
// past max_errors.
std::vector<Record> most_likely(const Plan& P, uint64_t k_max, const Criteria& crit) {
  std::vector<Item> items;
  for (size_t s = 0; s < P.sites.size(); ++s) {
    const double* p = &P.site_p[P.site_off[s]];
    int K = (int)(P.site_off[s + 1] - P.site_off[s]);
    for (int k = 1; k < K; ++k)
      if (p[k] > 0 && crit.allowed(s, k)) items.push_back({-std::log(p[k] / p[0]), (uint32_t)s, (uint8_t)k});
  }
  std::sort(items.begin(), items.end(), [](const Item& a, const Item& b) {
    if (a.c != b.c) return a.c < b.c;
    if (a.s != b.s) return a.s < b.s;
    return a.k < b.k;
  });
  std::vector<char> used(P.sites.size(), 0);
  // visit(tau, cap, sink): returns number of records with score <= tau (stops at cap)
  std::vector<uint32_t> stack_item;
  auto walk = [&](double tau, uint64_t cap, std::vector<std::pair<double, Record>>* sink) -> uint64_t {
    uint64_t count = 0;
    std::function<void(size_t, double)> rec_fn = [&](size_t start, double partial) {
      if (count >= cap) return;
      if (crit.keep(stack_item.size())) {
        ++count;
        if (sink) {
          Record r;
          for (uint32_t it : stack_item) r.push_back({items[it].s, items[it].k});
          std::sort(r.begin(), r.end());
          sink->push_back({partial, r});
        }
      }
      if (crit.max_errors && stack_item.size() >= crit.max_errors) return;
      for (size_t j = start; j < items.size(); ++j) {
        if (partial + items[j].c > tau) break;
        if (used[items[j].s]) continue;
        used[items[j].s] = 1;
        stack_item.push_back((uint32_t)j);
        rec_fn(j + 1, partial + items[j].c);
        stack_item.pop_back();
        used[items[j].s] = 0;
        if (count >= cap) return;
      }
    };
    rec_fn(0, 0.0);
    return count;
  };
  double tau;
  if (walk(0.0, k_max, nullptr) >= k_max) {
    tau = 0.0;
  } else {
    double total = 0.0;
    for (auto& it : items) total += it.c;
    double lo = 0.0, hi = items.empty() ? 0.0 : std::max(items.front().c, 1e-6);
    while (hi < total && walk(hi, k_max, nullptr) < k_max) {
      lo = hi;
      hi = std::min(total, hi * 2 + 1e-300);
    }
    if (walk(hi, k_max, nullptr) >= k_max) {
      for (int it = 0; it < 200 && hi > lo; ++it) {
        double mid = lo + (hi - lo) / 2;
        if (mid <= lo || mid >= hi) break;
        if (walk(mid, k_max, nullptr) >= k_max)
          hi = mid;
        else
          lo = mid;
      }
    }
    tau = hi;
  }
  std::vector<std::pair<double, Record>> all;
  walk(tau, std::numeric_limits<uint64_t>::max(), &all);
  std::sort(all.begin(), all.end(), [](const std::pair<double, Record>& a, const std::pair<double, Record>& b) {
    if (a.first != b.first) return a.first < b.first;
    return a.second < b.second;
  });
  std::vector<Record> out;
  for (size_t i = 0; i < all.size() && i < k_max; ++i) out.push_back(all[i].second);
  return out;
}

}  // namespace

// wbasis: the unnormalised ensemble weight of each record (see TrajSet::wbasis);
// empty = the records' counts.
static ptsbe_status make_trajset(std::shared_ptr<const Plan> plan, const std::vector<Record>& recs,
                                 std::vector<uint64_t> m, std::vector<uint64_t> counts, uint64_t alpha0,
                                 ptsbe_trajset_t* out, std::vector<double> wbasis = {}) {
  auto ts = std::make_shared<TrajSet>();
  ts->plan = plan;
  ts->alpha0 = alpha0;
  ts->rec_off.push_back(0);
  for (size_t a = 0; a < recs.size(); ++a) {
    for (auto& e : recs[a]) {
      ts->rec_site.push_back(e.first);
      ts->rec_kraus.push_back(e.second);
    }
    ts->rec_off.push_back((uint32_t)ts->rec_site.size());
    ts->p.push_back(joint_prob(*plan, recs[a]));
  }
  ts->m = std::move(m);
  ts->count = std::move(counts);
  if (wbasis.empty())
    for (auto v : ts->count) wbasis.push_back((double)v);
  ts->wbasis = std::move(wbasis);
  for (auto v : ts->m) ts->total_shots += v;
  for (auto v : ts->count) ts->total_count += v;
  auto* h = new (std::nothrow) ptsbe_trajset_s;
  if (!h) return fail(PTSBE_E_OOM, "host allocation failed");
  h->ts = ts;
  *out = h;
  return PTSBE_OK;
}

ptsbe_status sample_kraus(const std::shared_ptr<Plan>& plan, const ptsbe_pts_opts* o, ptsbe_trajset_t* out) {
  const Plan& P = *plan;
  const size_t S = P.sites.size();
  std::vector<Record> recs;
  std::vector<uint64_t> counts;
  uint64_t T = 0;
  Criteria crit;
  crit.P = &P;
  crit.allow = o->kraus_allow;
  crit.min_errors = o->min_errors;
  crit.max_errors = o->max_errors;
  crit.parity = o->error_parity;
  if (crit.parity > PTSBE_PARITY_ODD) return fail(PTSBE_E_ARG, "bad error parity");
  if (crit.max_errors && crit.min_errors > crit.max_errors) return fail(PTSBE_E_ARG, "min_errors > max_errors");
  if (o->mode == PTSBE_PTS_PROPORTIONAL || o->mode == PTSBE_PTS_PER_SHOT) {
    if (o->n_draws == 0 || o->n_draws > (1ull << 32)) return fail(PTSBE_E_ARG, "n_draws must be in 1..2^32");
    bool merge = o->mode == PTSBE_PTS_PROPORTIONAL;
    uint32_t stream = o->stream ? o->stream : (merge ? 1u : 3u);
    std::unordered_map<Record, size_t, RecordHash> index;
    T = o->n_draws;
    for (uint64_t t = 0; t < T; ++t) {
      uint64_t k1 = stream_key1(stream, o->cfg, t);
      Record rec;
      for (size_t s = 0; s < S; ++s) {
        double u = word_to_uniform(philox_word(o->seed, k1, s));
        int K = (int)(P.site_off[s + 1] - P.site_off[s]);
        int k = categorical(u, &P.site_p[P.site_off[s]], K);
        if (k && crit.allowed(s, k)) rec.push_back({(uint32_t)s, (uint8_t)k});
      }
      if (merge) {
        auto it = index.find(rec);
        if (it != index.end()) {
          counts[it->second] += 1;
          continue;
        }
        index.emplace(rec, recs.size());
      }
      recs.push_back(std::move(rec));
      counts.push_back(1);
    }
  } else if (o->mode == PTSBE_PTS_ALG2_LITERAL) {
    if (o->n_draws == 0 || o->n_draws > (1ull << 32)) return fail(PTSBE_E_ARG, "n_draws must be in 1..2^32");
    uint32_t stream = o->stream ? o->stream : 1u;
    std::unordered_map<Record, size_t, RecordHash> index;
    T = o->n_draws;
    for (uint64_t t = 0; t < T; ++t) {
      uint64_t k1 = stream_key1(stream, o->cfg, t);
      uint64_t j = 0;
      Record rec;
      for (size_t s = 0; s < S; ++s) {
        int K = (int)(P.site_off[s + 1] - P.site_off[s]);
        bool chosen = false;
        for (int k = 1; k < K; ++k) {
          double r = word_to_uniform(philox_word(o->seed, k1, j++));
          // compatible(): one per site; selection criteria: allowed operators only
          if (r <= P.site_p[P.site_off[s] + k] && !chosen && crit.allowed(s, k)) {
            rec.push_back({(uint32_t)s, (uint8_t)k});
            chosen = true;
          }
        }
      }
      auto it = index.find(rec);
      if (it != index.end()) {  // uniqueKraus()
        counts[it->second] += 1;
        continue;
      }
      index.emplace(rec, recs.size());
      recs.push_back(std::move(rec));
      counts.push_back(1);
    }
  } else if (o->mode == PTSBE_PTS_MOST_LIKELY) {
    if (o->k_max == 0 || o->k_max > (1ull << 26)) return fail(PTSBE_E_ARG, "k_max must be in 1..2^26");
    recs = most_likely(P, o->k_max, crit);
    counts.assign(recs.size(), 1);
    T = recs.size();
  } else {
    return fail(PTSBE_E_ARG, "unknown PTS mode");
  }
  // record-level selection criteria: drop the records (and their draws) that fail
  if (crit.any_filter() && o->mode != PTSBE_PTS_MOST_LIKELY) {
    std::vector<Record> r2;
    std::vector<uint64_t> c2;
    uint64_t T2 = 0;
    for (size_t a = 0; a < recs.size(); ++a)
      if (crit.keep(recs[a].size())) {
        r2.push_back(recs[a]);
        c2.push_back(counts[a]);
        T2 += counts[a];
      }
    recs.swap(r2);
    counts.swap(c2);
    T = T2;
  }
  if (recs.empty()) return fail(PTSBE_E_ARG, "no record meets the selection criteria");
  // probability band (Sec. 3.1): keep records with p_alpha in [p_min, p_max]
  if (o->p_min != 0.0 || o->p_max != 0.0) {
    if (!(o->p_min >= 0.0 && o->p_max >= o->p_min)) return fail(PTSBE_E_ARG, "bad probability band");
    std::vector<Record> r2;
    std::vector<uint64_t> c2;
    uint64_t T2 = 0;
    for (size_t a = 0; a < recs.size(); ++a) {
      double pa = joint_prob(P, recs[a]);
      if (pa >= o->p_min && pa <= o->p_max) {
        r2.push_back(recs[a]);
        c2.push_back(counts[a]);
        T2 += counts[a];
      }
    }
    recs.swap(r2);
    counts.swap(c2);
    T = T2;
    if (recs.empty()) return fail(PTSBE_E_ARG, "no record falls in the probability band");
  }
  // Shots and ensemble weights follow the allocation: draw counts (multiplicity),
  // joint probabilities (reweight), equal (uniform, one shot per draw).
  std::vector<uint64_t> m;
  std::vector<double> wb;
  if (o->mode == PTSBE_PTS_PER_SHOT) {
    m.assign(recs.size(), 1);
    wb.assign(recs.size(), 1.0);
  } else if (o->alloc == PTSBE_ALLOC_MULTIPLICITY) {
    if (o->mode == PTSBE_PTS_MOST_LIKELY) return fail(PTSBE_E_ARG, "most-likely mode uses REWEIGHT or UNIFORM");
    m = alloc_multiplicity(counts, T, o->total_shots);
    for (auto c : counts) wb.push_back((double)c);
  } else if (o->alloc == PTSBE_ALLOC_REWEIGHT) {
    for (auto& r : recs) wb.push_back(joint_prob(P, r));
    m = alloc_reweight(wb, o->total_shots);
  } else if (o->alloc == PTSBE_ALLOC_UNIFORM) {
    m.assign(recs.size(), o->nshots);
    wb.assign(recs.size(), 1.0);
  } else {
    return fail(PTSBE_E_ARG, "unknown allocation");
  }
  return make_trajset(plan, recs, std::move(m), std::move(counts), 0, out, std::move(wb));
}

ptsbe_status trajset_from_records(const std::shared_ptr<Plan>& plan, uint32_t n, const uint32_t* off,
                                  const uint32_t* site, const uint8_t* kraus, const uint64_t* m, uint64_t alpha0,
                                  ptsbe_trajset_t* out) {
  const Plan& P = *plan;
  if (n && (!off || !m)) return fail(PTSBE_E_ARG, "null record arrays");
  if (n && off[0] != 0) return fail(PTSBE_E_ARG, "rec_off[0] must be 0");
  std::vector<Record> recs(n);
  for (uint32_t a = 0; a < n; ++a) {
    if (off[a + 1] < off[a]) return fail(PTSBE_E_ARG, "rec_off must be non-decreasing");
    if (off[a + 1] > off[a] && (!site || !kraus)) return fail(PTSBE_E_ARG, "null record entries");
    for (uint32_t j = off[a]; j < off[a + 1]; ++j) {
      if (site[j] >= P.sites.size()) return fail(PTSBE_E_ARG, "record site out of range");
      uint32_t K = P.site_off[site[j] + 1] - P.site_off[site[j]];
      if (kraus[j] == 0 || kraus[j] >= K) return fail(PTSBE_E_ARG, "record Kraus index out of range");
      if (j > off[a] && site[j] <= site[j - 1]) return fail(PTSBE_E_ARG, "record sites must be ascending");
      recs[a].push_back({site[j], kraus[j]});
    }
  }
  std::vector<uint64_t> mm(m, m + n), cnt(n, 1);
  std::vector<double> wb;
  for (uint32_t a = 0; a < n; ++a) wb.push_back((double)m[a]);
  return make_trajset(plan, recs, std::move(mm), std::move(cnt), alpha0, out, std::move(wb));
}

ptsbe_status trajset_slice(const TrajSet& ts, uint32_t b, uint32_t e, ptsbe_trajset_t* out) {
  uint32_t n = (uint32_t)ts.m.size();
  if (b > e || e > n) return fail(PTSBE_E_ARG, "bad slice range");
  std::vector<Record> recs;
  for (uint32_t a = b; a < e; ++a) {
    Record r;
    for (uint32_t j = ts.rec_off[a]; j < ts.rec_off[a + 1]; ++j) r.push_back({ts.rec_site[j], ts.rec_kraus[j]});
    recs.push_back(r);
  }
  std::vector<uint64_t> m(ts.m.begin() + b, ts.m.begin() + e), c(ts.count.begin() + b, ts.count.begin() + e);
  std::vector<double> wb(ts.wbasis.begin() + b, ts.wbasis.begin() + e);
  return make_trajset(ts.plan, recs, std::move(m), std::move(c), ts.alpha0 + b, out, std::move(wb));
}

std::vector<double> ensemble_weights(const TrajSet& ts) {
  double tot = 0.0;
  for (double v : ts.wbasis) tot += v;
  std::vector<double> w(ts.wbasis.size(), 0.0);
  if (tot > 0.0)
    for (size_t a = 0; a < w.size(); ++a) w[a] = ts.wbasis[a] / tot;
  return w;
}

// ----------------------------------------------------------- device tables

static uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

template <typename T>
static void put(std::vector<uint8_t>& blob, uint64_t off, const T* src, size_t n) {
  if (n) std::memcpy(blob.data() + off, src, n * sizeof(T));
}

// Device tables of one fused program (forward or adjoint) for a trajectory set.
static void program_tables(const Plan& P, const std::vector<Step>& steps, const std::vector<Pass>& prog_passes,
                           const std::vector<ExecStep>& prog_exec,
                           const std::vector<std::vector<std::pair<int, int>>>& site_slots, const TrajSet& ts,
                           const std::vector<double>& pv, uint32_t chunk, std::vector<uint8_t>& blob_out,
                           TableLayout& L_out, std::vector<uint64_t>& chunk_off_out) {
  const uint32_t B = (uint32_t)ts.m.size();
  const uint32_t NP = (uint32_t)prog_passes.size();
  std::vector<DPass> passes(NP);
  std::vector<DOp> ops;
  std::vector<uint32_t> slot_default;
  std::vector<cd> pool;
  std::vector<uint32_t> slot_base(NP);
  std::map<int, int> empty;
  std::vector<std::vector<Mat>> defaults(NP);
  for (uint32_t p = 0; p < NP; ++p)
    for (const Slot& s : prog_passes[p].slots)
      defaults[p].push_back(slot_matrix(P, steps, s, pv.empty() ? nullptr : pv.data(), empty));
  const std::vector<std::vector<SlotFrame>> frames = slot_frames(P.n, prog_passes, prog_exec, defaults);
  for (uint32_t p = 0; p < NP; ++p) {
    const Pass& ps = prog_passes[p];
    DPass& d = passes[p];
    std::memset(&d, 0, sizeof(d));
    d.k = (uint32_t)ps.k;
    d.n_ops = (uint32_t)ps.ops.size();
    d.op_begin = (uint32_t)ops.size();
    d.slot_begin = (uint32_t)slot_default.size();
    d.n_slots = (uint32_t)ps.slots.size();
    d.flags = ps.flags;
    for (int j = 0; j < ps.k; ++j) d.tq[j] = (uint8_t)ps.tq[j];
    for (size_t j = 0; j < ps.oq.size(); ++j) d.oq[j] = (uint8_t)ps.oq[j];
    ops.insert(ops.end(), ps.ops.begin(), ps.ops.end());
    slot_base[p] = (uint32_t)slot_default.size();
    for (size_t si = 0; si < ps.slots.size(); ++si) {
      const Mat M = frame_matrix(ps.slots[si], frames[p][si], defaults[p][si]);
      slot_default.push_back((uint32_t)pool.size());
      pool.insert(pool.end(), M.begin(), M.end());
    }
  }
  // per-trajectory overrides
  std::vector<uint32_t> ov_off((size_t)B * NP + 1, 0);
  std::vector<DOverride> ov;
  std::map<std::pair<std::pair<int, int>, std::vector<std::pair<int, int>>>, uint32_t> dedupe;
  for (uint32_t a = 0; a < B; ++a) {
    std::map<std::pair<int, int>, std::map<int, int>> touched;  // (pass, slot) -> site choices
    for (uint32_t j = ts.rec_off[a]; j < ts.rec_off[a + 1]; ++j) {
      int site = (int)ts.rec_site[j];
      for (auto& ps : site_slots[site]) touched[ps][site] = ts.rec_kraus[j];
    }
    std::vector<std::vector<DOverride>> per_pass(NP);
    for (auto& kv : touched) {
      int p = kv.first.first, s = kv.first.second;
      std::vector<std::pair<int, int>> key(kv.second.begin(), kv.second.end());
      auto dk = std::make_pair(kv.first, key);
      auto it = dedupe.find(dk);
      uint32_t off;
      if (it != dedupe.end()) {
        off = it->second;
      } else {
        const Slot& sl = prog_passes[p].slots[s];
        const Mat M = frame_matrix(sl, frames[p][s], slot_matrix(P, steps, sl, pv.empty() ? nullptr : pv.data(),
                                                                  kv.second));
        off = (uint32_t)pool.size();
        pool.insert(pool.end(), M.begin(), M.end());
        dedupe.emplace(dk, off);
      }
      per_pass[p].push_back({(uint32_t)s, off});
    }
    for (uint32_t p = 0; p < NP; ++p) {
      ov_off[(size_t)a * NP + p] = (uint32_t)ov.size();
      ov.insert(ov.end(), per_pass[p].begin(), per_pass[p].end());
    }
  }
  ov_off[(size_t)B * NP] = (uint32_t)ov.size();
  std::vector<uint64_t> shot_off(B + 1, 0), chunk_off(B + 1, 0);
  for (uint32_t a = 0; a < B; ++a) {
    shot_off[a + 1] = shot_off[a] + ts.m[a];
    chunk_off[a + 1] = chunk_off[a] + (ts.m[a] + chunk - 1) / chunk;
  }
  // layout
  const bool c64 = P.precision == PTSBE_C64;
  const size_t esz = c64 ? 8 : 16;
  TableLayout L{};
  uint64_t o = 0;
  L.passes = o; o = align256(o + passes.size() * sizeof(DPass));
  L.ops = o; o = align256(o + std::max<size_t>(1, ops.size()) * sizeof(DOp));
  L.slot_default = o; o = align256(o + std::max<size_t>(1, slot_default.size()) * 4);
  L.pool = o; o = align256(o + std::max<size_t>(1, pool.size()) * esz);
  L.ov_off = o; o = align256(o + ov_off.size() * 4);
  L.ov = o; o = align256(o + std::max<size_t>(1, ov.size()) * sizeof(DOverride));
  L.shot_off = o; o = align256(o + shot_off.size() * 8);
  L.chunk_off = o; o = align256(o + chunk_off.size() * 8);
  std::vector<DExec> exec(prog_exec.size());
  for (size_t e = 0; e < prog_exec.size(); ++e) {
    DExec& d = exec[e];
    std::memset(&d, 0, sizeof(d));
    const ExecStep& ex = prog_exec[e];
    d.pass = ex.pass >= 0 ? (uint32_t)ex.pass : 0xffffffffu;
    d.nq = (uint32_t)std::min<size_t>(16, ex.mr_qubits.size());
    for (uint32_t j = 0; j < d.nq; ++j) {
      d.q[j] = (uint32_t)ex.mr_qubits[j];
      d.idx[j] = (uint32_t)ex.mr_index[j];
    }
  }
  L.exec = o; o = align256(o + std::max<size_t>(1, exec.size()) * sizeof(DExec));
  L.total = o;
  L.n_passes = passes.size();
  L.n_ops = ops.size();
  L.n_slots = slot_default.size();
  L.n_pool = pool.size();
  L.n_ov = ov.size();
  L.n_exec = exec.size();
  std::vector<uint8_t> blob(L.total, 0);
  put(blob, L.passes, passes.data(), passes.size());
  put(blob, L.ops, ops.data(), ops.size());
  put(blob, L.slot_default, slot_default.data(), slot_default.size());
  if (c64) {
    std::vector<float> f(pool.size() * 2);
    for (size_t i = 0; i < pool.size(); ++i) {
      f[2 * i] = (float)pool[i].real();
      f[2 * i + 1] = (float)pool[i].imag();
    }
    put(blob, L.pool, f.data(), f.size());
  } else {
    std::vector<double> f(pool.size() * 2);
    for (size_t i = 0; i < pool.size(); ++i) {
      f[2 * i] = pool[i].real();
      f[2 * i + 1] = pool[i].imag();
    }
    put(blob, L.pool, f.data(), f.size());
  }
  put(blob, L.ov_off, ov_off.data(), ov_off.size());
  put(blob, L.ov, ov.data(), ov.size());
  put(blob, L.shot_off, shot_off.data(), shot_off.size());
  put(blob, L.chunk_off, chunk_off.data(), chunk_off.size());
  put(blob, L.exec, exec.data(), exec.size());
  blob_out.swap(blob);
  L_out = L;
  chunk_off_out = chunk_off;
}

ptsbe_status build_tables(TrajSet& ts, const double* params, uint32_t chunk) {
  const Plan& P = *ts.plan;
  std::vector<double> pv(params ? params : nullptr, params ? params + P.n_params : nullptr);
  if (ts.table_valid && pv == ts.cached_params && chunk == ts.cached_chunk) return PTSBE_OK;
  program_tables(P, P.steps, P.passes, P.exec, P.site_slots, ts, pv, chunk, ts.table_blob, ts.layout, ts.chunk_off);
  ts.cached_params = pv;
  ts.cached_chunk = chunk;
  ts.table_valid = true;
  return PTSBE_OK;
}

ptsbe_status build_adj_tables(TrajSet& ts, const double* params) {
  const Plan& P = *ts.plan;
  if (!P.has_adjoint) return fail(PTSBE_E_UNSUPPORTED, "no adjoint program (no parameters, or measure-reset/projection)");
  std::vector<double> pv(params ? params : nullptr, params ? params + P.n_params : nullptr);
  if (ts.adj_valid && pv == ts.adj_params) return PTSBE_OK;
  std::vector<uint64_t> chunk_off;
  program_tables(P, P.adj.steps, P.adj.passes, P.adj.exec, P.adj.site_slots, ts, pv, 4096, ts.adj_blob,
                 ts.adj_layout, chunk_off);
  ts.adj_params = pv;
  ts.adj_valid = true;
  return PTSBE_OK;
}

}  // namespace ptsbe
