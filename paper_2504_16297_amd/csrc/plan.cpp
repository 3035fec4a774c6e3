// Plan construction: validation of the noisy circuit, unitary-mixture analysis
// of every channel (Sec. 2.2), expansion into noise sites (the NoisyCircuit of
// Algorithm 2), and fusion of the operations into LDS tile passes.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <set>
#include <sstream>

#include "host.hpp"
#include "jit.hpp"

namespace ptsbe {

static thread_local std::string g_last_error;

ptsbe_status fail(ptsbe_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

const char* last_error_cstr() { return g_last_error.c_str(); }

Mat mat_identity(int d) {
  Mat m(d * d, cd(0, 0));
  for (int i = 0; i < d; ++i) m[i * d + i] = 1.0;
  return m;
}

Mat mat_mul(const Mat& a, const Mat& b, int d) {
  Mat c(d * d, cd(0, 0));
  for (int i = 0; i < d; ++i)
    for (int k = 0; k < d; ++k) {
      cd aik = a[i * d + k];
      if (aik == cd(0, 0)) continue;
      for (int j = 0; j < d; ++j) c[i * d + j] += aik * b[k * d + j];
    }
  return c;
}

bool mat_is_diag(const Mat& a, int d, double tol) {
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j)
      if (i != j && std::abs(a[i * d + j]) > tol) return false;
  return true;
}

Mat rot_matrix(int gen, double theta) {
  double c = std::cos(theta / 2), s = std::sin(theta / 2);
  Mat m(4);
  if (gen == PTSBE_GEN_X) {
    m = {cd(c, 0), cd(0, -s), cd(0, -s), cd(c, 0)};
  } else if (gen == PTSBE_GEN_Y) {
    m = {cd(c, 0), cd(-s, 0), cd(s, 0), cd(c, 0)};
  } else {
    m = {cd(c, -s), cd(0, 0), cd(0, 0), cd(c, s)};
  }
  return m;
}

static Mat read_mat(const double* p, int d) {
  Mat m(d * d);
  for (int i = 0; i < d * d; ++i) m[i] = cd(p[2 * i], p[2 * i + 1]);
  return m;
}

// tr(K^dagger K)/d, element by element in row-major order.
static double kraus_weight(const Mat& K, int d) {
  double s = 0.0;
  for (int i = 0; i < d * d; ++i) s += K[i].real() * K[i].real() + K[i].imag() * K[i].imag();
  return s / d;
}

// U = A (x) B with A on matrix bit 1 and B on bit 0?  Fills a, b when so.
static bool split_product(const Mat& U, Mat* a, Mat* b) {
  // R[(r1 c1), (r0 c0)] = U[2 r1 + r0][2 c1 + c0] must be rank one.
  cd R[4][4];
  for (int r1 = 0; r1 < 2; ++r1)
    for (int c1 = 0; c1 < 2; ++c1)
      for (int r0 = 0; r0 < 2; ++r0)
        for (int c0 = 0; c0 < 2; ++c0) R[r1 * 2 + c1][r0 * 2 + c0] = U[(2 * r1 + r0) * 4 + 2 * c1 + c0];
  int bi = 0, bj = 0;
  double best = -1;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      if (std::abs(R[i][j]) > best) {
        best = std::abs(R[i][j]);
        bi = i;
        bj = j;
      }
  if (best <= 0) return false;
  Mat A(4), B(4);
  for (int i = 0; i < 4; ++i) A[i] = R[i][bj];
  for (int j = 0; j < 4; ++j) B[j] = R[bi][j] / R[bi][bj];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      if (std::abs(R[i][j] - A[i] * B[j]) > 1e-12) return false;
  // A[r1*2+c1] is the 2x2 on bit 1; B[r0*2+c0] on bit 0.
  *a = A;
  *b = B;
  return true;
}

// ------------------------------------------------------------ Pauli twirl

// Pauli string `index` on nq qubits: base-4 digit j (0 I, 1 X, 2 Y, 3 Z) acts
// on matrix bit j.
static Mat pauli_matrix(uint32_t index, int nq) {
  static const cd s[4][4] = {{1, 0, 0, 1}, {0, 1, 1, 0}, {0, cd(0, -1), cd(0, 1), 0}, {1, 0, 0, -1}};
  const int d = 1 << nq;
  Mat M(d * d);
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c) {
      cd v(1, 0);
      for (int j = 0; j < nq; ++j) v *= s[(index >> (2 * j)) & 3][((r >> j) & 1) * 2 + ((c >> j) & 1)];
      M[r * d + c] = v;
    }
  return M;
}

// Averaging a channel over conjugation by every Pauli string keeps the diagonal
// of its Pauli transfer matrix: the Pauli channel with p_P = sum_k |Tr(P^dag K_k)|^2 / d^2.
std::vector<double> pauli_twirl_probs(const std::vector<Mat>& K, int nq) {
  const int d = 1 << nq;
  std::vector<double> p(d * d, 0.0);
  for (uint32_t i = 0; i < (uint32_t)(d * d); ++i) {
    const Mat P = pauli_matrix(i, nq);
    for (const Mat& m : K) {
      cd tr(0, 0);
      for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) tr += std::conj(P[r * d + c]) * m[r * d + c];
      p[i] += std::norm(tr) / (double)(d * d);
    }
  }
  return p;
}

ptsbe_status pauli_twirl_channel(uint32_t nq, const double* kraus, uint32_t n_kraus, double* probs) {
  if (nq < 1 || nq > 2 || n_kraus < 1 || n_kraus > 64 || !kraus || !probs)
    return fail(PTSBE_E_ARG, "Pauli twirl: nq 1 or 2, 1..64 Kraus operators, non-null arrays");
  const int d = 1 << nq;
  std::vector<Mat> K;
  for (uint32_t k = 0; k < n_kraus; ++k) K.push_back(read_mat(kraus + 2 * k * d * d, d));
  double err = 0;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      cd v(0, 0);
      for (auto& m : K)
        for (int l = 0; l < d; ++l) v += std::conj(m[l * d + i]) * m[l * d + j];
      err = std::max(err, std::abs(v - (i == j ? 1.0 : 0.0)));
    }
  if (err > 1e-12) return fail(PTSBE_E_NOT_CPTP, "Pauli twirl: the channel is not CPTP");
  const std::vector<double> p = pauli_twirl_probs(K, (int)nq);
  std::copy(p.begin(), p.end(), probs);
  return PTSBE_OK;
}

static ptsbe_status analyse_channel(const ptsbe_channel& ch, int idx, Channel* out, bool twirl = false) {
  if (ch.nq < 1 || ch.nq > 2) return fail(PTSBE_E_ARG, "channel " + std::to_string(idx) + ": nq must be 1 or 2");
  if (ch.n_kraus < 1 || ch.n_kraus > 16 || !ch.kraus)
    return fail(PTSBE_E_ARG, "channel " + std::to_string(idx) + ": 1..16 Kraus operators required");
  int d = 1 << ch.nq;
  Channel c;
  c.nq = ch.nq;
  c.K = ch.n_kraus;
  std::vector<Mat> K;
  for (uint32_t k = 0; k < ch.n_kraus; ++k) K.push_back(read_mat(ch.kraus + 2 * k * d * d, d));
  // CPTP: sum_k K^dagger K = I (Sec. 2.2)
  Mat acc(d * d, cd(0, 0));
  for (auto& m : K)
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j)
        for (int l = 0; l < d; ++l) acc[i * d + j] += std::conj(m[l * d + i]) * m[l * d + j];
  double err = 0;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) err = std::max(err, std::abs(acc[i * d + j] - (i == j ? 1.0 : 0.0)));
  if (err > 1e-12) {
    std::ostringstream os;
    os << "channel " << idx << " is not CPTP: max |sum K^dag K - I| = " << err;
    return fail(PTSBE_E_NOT_CPTP, os.str());
  }
  // unitary mixture: K^dagger K = p I (Sec. 2.2 feature 2)
  c.all_diag = true;
  for (int k = 0; k < c.K; ++k) {
    double p = kraus_weight(K[k], d);
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        cd v(0, 0);
        for (int l = 0; l < d; ++l) v += std::conj(K[k][l * d + i]) * K[k][l * d + j];
        if (std::abs(v - (i == j ? p : 0.0)) > 1e-12) {
          if (!twirl) {
            // Not a unitary mixture: resolved when the trajectory's state reaches
            // it (Algorithm 1's state-dependent branch, p_k = <psi|K_k^dag K_k|psi>).
            // A 1-qubit channel with diagonal K_k^dagger K_k needs only the qubit's
            // populations and is applied inside the next tile pass; any other
            // (dense: a 1-qubit channel with non-diagonal K^dag K, or a 2-qubit
            // channel) needs the reduced density matrix of its qubits and is
            // applied by its own step.
            Channel g;
            g.nq = ch.nq;
            g.K = ch.n_kraus;
            g.general = true;
            g.dense = ch.nq != 1;
            for (int kk = 0; kk < g.K; ++kk) {
              Mat m(d * d, cd(0, 0));
              for (int r = 0; r < d; ++r)
                for (int c2 = 0; c2 < d; ++c2)
                  for (int l = 0; l < d; ++l) m[r * d + c2] += std::conj(K[kk][l * d + r]) * K[kk][l * d + c2];
              if (d == 2) {
                if (std::abs(m[1]) > 1e-12 || std::abs(m[2]) > 1e-12) g.dense = true;
                g.d0.push_back(m[0].real());
                g.d1.push_back(m[3].real());
              }
              g.M.push_back(m);
              g.U.push_back(K[kk]);
              g.p.push_back(kraus_weight(K[kk], d));
              g.diag.push_back(mat_is_diag(K[kk], d));
            }
            *out = std::move(g);
            return PTSBE_OK;
          }
          // its Pauli twirl: sqrt(p_P) P for the strings with p_P > 0, in string order
          const std::vector<double> pt = pauli_twirl_probs(K, ch.nq);
          std::vector<double> flat;
          uint32_t nk = 0;
          for (uint32_t s = 0; s < pt.size(); ++s) {
            if (pt[s] <= 0.0) continue;
            const Mat P = pauli_matrix(s, ch.nq);
            for (const cd& x : P) {
              flat.push_back(x.real() * std::sqrt(pt[s]));
              flat.push_back(x.imag() * std::sqrt(pt[s]));
            }
            ++nk;
          }
          ptsbe_channel tw = ch;
          tw.n_kraus = nk;
          tw.kraus = flat.data();
          return analyse_channel(tw, idx, out, false);
        }
      }
    Mat U = K[k];
    if (p > 0) {
      double s = 1.0 / std::sqrt(p);
      for (auto& x : U) x *= s;
    } else {
      U = mat_identity(d);
    }
    c.p.push_back(p);
    bool dg = mat_is_diag(U, d);
    c.diag.push_back(dg);
    c.all_diag = c.all_diag && dg;
    c.U.push_back(U);
  }
  if (c.nq == 2) {
    c.product = true;
    for (int k = 0; k < c.K; ++k) {
      Mat a, b;
      if (!split_product(c.U[k], &a, &b)) {
        c.product = false;
        break;
      }
      c.f1.push_back(a);
      c.f0.push_back(b);
    }
    if (!c.product) {
      c.f0.clear();
      c.f1.clear();
    }
  }
  *out = std::move(c);
  return PTSBE_OK;
}

// ------------------------------------------------------------------ fusion

static Mat mat_dagger(const Mat& a) {
  const int d = a.size() == 16 ? 4 : 2;
  Mat r(a.size());
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) r[i * d + j] = std::conj(a[j * d + i]);
  return r;
}

static Mat part_matrix(const Plan& plan, const std::vector<Step>& steps, const Part& pt, const double* params,
                       const std::map<int, int>& choice) {
  const Step& st = steps[pt.step];
  Mat m;
  switch (st.kind) {
    case ST_GATE:
    case ST_P0:
      m = st.mat;
      break;
    case ST_PARAM:
      m = rot_matrix(st.gen, params ? params[st.param] : 0.0);
      break;
    case ST_SITE: {
      const Site& s = plan.sites[st.site];
      const Channel& ch = plan.channels[s.channel];
      auto it = choice.find(st.site);
      int k = it == choice.end() ? 0 : it->second;
      if (pt.half < 0)
        m = ch.U[k];
      else
        m = pt.half == 0 ? ch.f0[k] : ch.f1[k];
      break;
    }
    default:
      return mat_identity(2);
  }
  return st.dagger ? mat_dagger(m) : m;
}

Mat slot_matrix(const Plan& plan, const std::vector<Step>& steps, const Slot& s, const double* params,
                const std::map<int, int>& choice) {
  if (s.type == DOP_KR) {  // the channel's Kraus operators, 4 entries each
    const Channel& c = plan.channels[steps[s.parts[0].step].chan];
    Mat M;
    for (const Mat& k : c.U) M.insert(M.end(), k.begin(), k.end());
    return M;
  }
  int d = (s.type == DOP_M2 || s.type == DOP_D2) ? 4 : 2;
  Mat M = mat_identity(d);
  for (const Part& pt : s.parts) {
    Mat m = part_matrix(plan, steps, pt, params, choice);
    if (pt.emb == 0 || pt.emb == 1) {
      // 2x2 on matrix bit emb of the 4x4: index bit 0 is the slot's first qubit
      Mat e(16, cd(0, 0));
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          const int ib = (i >> pt.emb) & 1, jb = (j >> pt.emb) & 1;
          const int io = (i >> (1 - pt.emb)) & 1, jo = (j >> (1 - pt.emb)) & 1;
          if (io == jo) e[i * 4 + j] = m[ib * 2 + jb];
        }
      m = e;
    } else if (pt.emb == 2) {
      // swap the two matrix bits: index (b1 b0) -> (b0 b1)
      auto sw = [](int x) { return ((x & 1) << 1) | ((x >> 1) & 1); };
      Mat e(16);
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) e[sw(i) * 4 + sw(j)] = m[i * 4 + j];
      m = e;
    }
    M = mat_mul(m, M, d);
  }
  return M;
}

namespace {

struct Fuser {
  Plan& plan;
  const std::vector<Step>& steps;
  Pass& pass;
  std::vector<int> run;  // qubit -> open slot index or -1
  std::vector<int> local;

  Fuser(Plan& pl, const std::vector<Step>& st, Pass& ps)
      : plan(pl), steps(st), pass(ps), run(pl.n, -1), local(pl.n, -1) {
    for (int j = 0; j < ps.k; ++j) local[ps.tq[j]] = j;
  }

  int new_slot(uint8_t type, int q0, int q1) {
    Slot s;
    s.type = type;
    s.q[0] = q0;
    s.q[1] = q1;
    pass.slots.push_back(s);
    return (int)pass.slots.size() - 1;
  }

  void add_part(int slot, const Part& pt) {
    Slot& s = pass.slots[slot];
    s.parts.push_back(pt);
    const Step& st = steps[pt.step];
    if (st.kind == ST_SITE) {
      if (std::find(s.sites.begin(), s.sites.end(), st.site) == s.sites.end()) s.sites.push_back(st.site);
    }
    if (st.kind == ST_PARAM) s.uses_params = true;
  }

  void emit(int slot) {
    Slot& s = pass.slots[slot];
    DOp op{};
    op.type = s.type;
    op.slot[0] = (uint16_t)slot;
    if (s.type == DOP_M1) {
      op.a = (uint8_t)local[s.q[0]];
    } else if (s.type == DOP_M2) {
      op.a = (uint8_t)local[s.q[0]];
      op.b = (uint8_t)local[s.q[1]];
    } else if (s.type == DOP_D1) {
      op.ga = (uint8_t)s.q[0];
      op.a = local[s.q[0]] >= 0 ? (uint8_t)local[s.q[0]] : (uint8_t)255;
    } else {
      op.ga = (uint8_t)s.q[0];
      op.gb = (uint8_t)s.q[1];
      op.a = local[s.q[0]] >= 0 ? (uint8_t)local[s.q[0]] : (uint8_t)255;
      op.b = local[s.q[1]] >= 0 ? (uint8_t)local[s.q[1]] : (uint8_t)255;
    }
    pass.ops.push_back(op);
  }

  void flush(int q) {
    const int s = run[q];
    if (s >= 0) {
      emit(s);
      run[q] = -1;
      if (pass.slots[s].type == DOP_M2) run[pass.slots[s].q[0] == q ? pass.slots[s].q[1] : pass.slots[s].q[0]] = -1;
    }
  }

  void one_qubit(int q, Part pt) {
    if (run[q] < 0) run[q] = new_slot(local[q] >= 0 ? DOP_M1 : DOP_D1, q, -1);
    const Slot& s = pass.slots[run[q]];
    if (s.type == DOP_M2) pt.emb = s.q[0] == q ? 0 : 1;
    add_part(run[q], pt);
  }

  // Pair fusion: a diagonal 2-qubit operation whose qubits both hold an open
  // 2x2 run (in the tile) turns the run of its first qubit into a 4x4 slot that
  // takes the other run, the operation, and the following 1-qubit operations
  // on either qubit; the other run's slot is left empty and dropped at finish.
  bool fuse_pair(int si) {
    const Step& st = steps[si];
    const int a = st.q[0], b = st.q[1];
    if (!plan.pair_fusion || !st.diag || local[a] < 0 || local[b] < 0) return false;
    if (run[a] < 0 || run[b] < 0 || run[a] == run[b]) return false;
    Slot& sa = pass.slots[run[a]];
    Slot& sb = pass.slots[run[b]];
    if (sa.type != DOP_M1 || sb.type != DOP_M1) return false;
    sa.type = DOP_M2;
    sa.q[1] = b;
    for (Part& pt : sa.parts) pt.emb = 0;
    for (Part pt : sb.parts) {
      pt.emb = 1;
      add_part(run[a], pt);
    }
    sb.parts.clear();
    sb.sites.clear();
    sb.uses_params = false;
    add_part(run[a], Part{si, -1});
    run[b] = run[a];
    return true;
  }

  void take(int si) {
    const Step& st = steps[si];
    if (st.kind == ST_DOT) {
      // gradient contribution Im<lambda|P_q|psi> at this point of the reverse sweep
      flush(st.q[0]);
      DOp op{};
      op.type = DOP_DOT;
      op.a = (uint8_t)local[st.q[0]];
      op.b = (uint8_t)st.gen;
      op.slot[0] = (uint16_t)(st.dot & 0xffff);
      op.slot[1] = (uint16_t)(st.dot >> 16);
      pass.ops.push_back(op);
      return;
    }
    if (st.kind == ST_MR) {
      flush(st.q[0]);
      DOp op{};
      op.type = DOP_MR;
      op.a = (uint8_t)local[st.q[0]];
      op.slot[0] = (uint16_t)st.mr;
      pass.ops.push_back(op);
      return;
    }
    if (st.kind == ST_GCH) {
      // K_k / sqrt(p_k) with k decided on the device; the slot holds K_0..K_{K-1}
      flush(st.q[0]);
      const int s = new_slot(DOP_KR, st.q[0], -1);
      add_part(s, Part{si, -1});
      DOp op{};
      op.type = DOP_KR;
      op.a = (uint8_t)local[st.q[0]];
      op.slot[0] = (uint16_t)st.mr;
      op.slot[1] = (uint16_t)s;
      pass.ops.push_back(op);
      return;
    }
    if (st.nq == 1) {
      one_qubit(st.q[0], Part{si, -1});
      return;
    }
    if (st.kind == ST_SITE) {
      const Channel& ch = plan.channels[plan.sites[st.site].channel];
      if (ch.product) {
        one_qubit(st.q[0], Part{si, 0});
        one_qubit(st.q[1], Part{si, 1});
        return;
      }
    }
    // 2-qubit operation: into the open 4x4 slot of exactly its two qubits, or
    // merged with the 2x2 runs on them, or a slot of its own
    if (run[st.q[0]] >= 0 && run[st.q[0]] == run[st.q[1]]) {
      const Slot& sl = pass.slots[run[st.q[0]]];
      add_part(run[st.q[0]], Part{si, -1, sl.q[0] == st.q[0] ? -1 : 2});
      return;
    }
    if (fuse_pair(si)) return;
    flush(st.q[0]);
    flush(st.q[1]);
    int s = new_slot(st.diag ? DOP_D2 : DOP_M2, st.q[0], st.q[1]);
    add_part(s, Part{si, -1});
    emit(s);
  }

  void finish() {
    for (int q = 0; q < plan.n; ++q) flush(q);
    // drop slots no operation refers to (runs taken over by pair fusion)
    std::vector<int> remap(pass.slots.size(), -1);
    auto slot_ref = [](DOp& op) -> uint16_t* {
      switch (op.type) {
        case DOP_M1:
        case DOP_M2:
        case DOP_D1:
        case DOP_D2: return &op.slot[0];
        case DOP_KR: return &op.slot[1];
        default: return nullptr;
      }
    };
    for (DOp& op : pass.ops)
      if (uint16_t* r = slot_ref(op)) remap[*r] = 0;
    std::vector<Slot> kept;
    for (size_t i = 0; i < pass.slots.size(); ++i)
      if (remap[i] == 0) {
        remap[i] = (int)kept.size();
        kept.push_back(pass.slots[i]);
      }
    if (kept.size() == pass.slots.size()) return;
    pass.slots.swap(kept);
    for (DOp& op : pass.ops)
      if (uint16_t* r = slot_ref(op)) *r = (uint16_t)remap[*r];
  }
};

}  // namespace

// Diagonal slots made of one fixed gate whose entries are all +-1 (CZ, Z, ...)
// become sign ops: the kernels flip signs instead of multiplying by phases.
static void lower_signs(const std::vector<Step>& steps, Pass& ps) {
  for (DOp& op : ps.ops) {
    if (op.type != DOP_D1 && op.type != DOP_D2) continue;
    const Slot& s = ps.slots[op.slot[0]];
    if (s.parts.size() != 1 || !s.sites.empty() || s.uses_params) continue;
    const Step& st = steps[s.parts[0].step];
    if (st.kind != ST_GATE && st.kind != ST_P0) continue;
    const int d = op.type == DOP_D1 ? 2 : 4;
    uint16_t mask = 0;
    bool ok = true;
    for (int i = 0; i < d; ++i) {
      cd v = st.mat[i * d + i];
      if (v == cd(1, 0)) continue;
      if (v == cd(-1, 0)) {
        mask |= (uint16_t)(1u << i);
        continue;
      }
      ok = false;
    }
    if (!ok) continue;
    if (op.type == DOP_D1) {
      op.b = 254;
      op.gb = 0;
    }
    op.type = DOP_DSIGN;
    op.slot[0] = mask;
  }
}

static bool is_diag_op(const DOp& op) { return op.type == DOP_D1 || op.type == DOP_D2 || op.type == DOP_DSIGN; }

static int op_qubits(const Pass& ps, const DOp& op, int* q) {
  switch (op.type) {
    case DOP_M1:
    case DOP_MR:
    case DOP_KR:
    case DOP_DOT:
      q[0] = ps.tq[op.a];
      return 1;
    case DOP_M2:
      q[0] = ps.tq[op.a];
      q[1] = ps.tq[op.b];
      return 2;
    case DOP_D1:
      q[0] = op.ga;
      return 1;
    case DOP_D2:
      q[0] = op.ga;
      q[1] = op.gb;
      return 2;
    case DOP_DSIGN:
      q[0] = op.ga;
      if (op.b == 254) return 1;
      q[1] = op.gb;
      return 2;
    default:
      return 0;
  }
}

// Order the pass's operations into register phases for the register kernel:
// each thread holds 2^kRegBits amplitudes spanning kRegBits local bits; an
// operation runs when its local bits are register bits (diagonal operations run
// anywhere).  A DOP_PHASE op switches the register bits through LDS.  Any
// topological order of the dependency graph (operations sharing a qubit, unless
// both are diagonal) is valid; the greedy walk below keeps phases few.  The pass
// starts and ends with the top kRegBits local bits in registers so that global
// loads and stores keep the lowest local bits across lanes.
static void schedule_phases(Pass& ps, int min_fill) {
  const int k = ps.k;
  if (k < (int)kMinRegTile) return;
  const int nops = (int)ps.ops.size();
  const int identity_slot = (int)ps.slots.size();  // 2x2 identity for idle register positions
  {
    Slot idn;
    idn.type = DOP_M1;
    idn.q[0] = idn.q[1] = -1;
    ps.slots.push_back(idn);
  }
  std::vector<std::vector<int>> preds(nops);
  for (int i = 0; i < nops; ++i) {
    int qi[2];
    int ni = op_qubits(ps, ps.ops[i], qi);
    for (int j = 0; j < i; ++j) {
      if (is_diag_op(ps.ops[i]) && is_diag_op(ps.ops[j])) continue;
      int qj[2];
      int nj = op_qubits(ps, ps.ops[j], qj);
      bool share = false;
      for (int x = 0; x < ni; ++x)
        for (int y = 0; y < nj; ++y) share = share || qi[x] == qj[y];
      if (share) preds[i].push_back(j);
    }
  }
  std::vector<char> done(nops, 0);
  int ndone = 0;
  std::vector<int> R_io;
  for (int j = k - (int)kRegBits; j < k; ++j) R_io.push_back(j);
  std::vector<int> R = R_io;
  auto inR = [&](int bit) { return std::find(R.begin(), R.end(), bit) != R.end(); };
  auto ready = [&](int i) {
    for (int p : preds[i])
      if (!done[p]) return false;
    return true;
  };
  // register bits an operation needs (a 4x4 matrix both of its bits: the
  // compiled kernels then apply it in registers)
  auto local_bits = [&](const DOp& op, int* b) -> int {
    if (op.type == DOP_M1 || op.type == DOP_MR || op.type == DOP_KR || op.type == DOP_DOT) {
      b[0] = op.a;
      return 1;
    }
    if (op.type == DOP_M2) {
      b[0] = op.a;
      b[1] = op.b;
      return 2;
    }
    return 0;
  };
  auto fits = [&](const DOp& op) {
    int b[2];
    int nb = local_bits(op, b);
    for (int x = 0; x < nb; ++x)
      if (!inR(b[x])) return false;
    return true;
  };
  auto phase_op = [](const std::vector<int>& r) {
    DOp op{};
    op.type = DOP_PHASE;
    op.a = (uint8_t)r[0];
    op.b = (uint8_t)r[1];
    op.ga = (uint8_t)r[2];
    op.gb = (uint8_t)r[3];
    return op;
  };
  std::vector<DOp> out;
  bool force_wave = false;  // the last register change brought nothing new: run the waves there are
  while (ndone < nops) {
    // Waves: every operation ready at the start of a wave is independent of the
    // others in it.  The wave's 2x2 matrices (at most one per register position)
    // become one M1G op, run as straight-line code on all 16 amplitudes.
    while (true) {
      std::vector<int> wave;
      for (int i = 0; i < nops; ++i)
        if (!done[i] && ready(i) && fits(ps.ops[i])) wave.push_back(i);
      if (wave.empty()) break;
      // A wave with few 2x2 matrices leaves register positions idle; when other
      // tile bits hold at least min_fill ready ones, emit only its diagonal ops
      // and switch registers instead.
      int m1_here = 0, m1_other = 0, reg_others = 0;
      for (int i = 0; i < nops; ++i)
        if (!done[i] && ready(i) && (ps.ops[i].type == DOP_M1 || ps.ops[i].type == DOP_M2))
          (fits(ps.ops[i]) ? m1_here : m1_other) += ps.ops[i].type == DOP_M2 ? 2 : 1;
      for (int i : wave)  // measure-resets and gradient terms in registers: never put off
        if (ps.ops[i].type == DOP_MR || ps.ops[i].type == DOP_KR || ps.ops[i].type == DOP_DOT) ++reg_others;
      if (!force_wave && reg_others == 0 && m1_here > 0 && m1_here < min_fill &&
          std::min(m1_other, (int)kRegBits) >= min_fill) {
        std::vector<int> diag;
        bool any_sign = false;
        for (int i : wave)
          if (is_diag_op(ps.ops[i])) diag.push_back(i);
        for (int i : diag) {
          out.push_back(ps.ops[i]);
          any_sign = any_sign || ps.ops[i].type == DOP_DSIGN;
          done[i] = 1;
          ++ndone;
        }
        if (any_sign) {
          DOp f{};
          f.type = DOP_SFLIP;
          out.push_back(f);
        }
        if (diag.empty()) break;
        continue;
      }
      DOp g{};
      g.type = DOP_M1G;
      for (int i : wave) {
        const DOp& op = ps.ops[i];
        if (op.type == DOP_M1) {
          const int j = (int)(std::find(R.begin(), R.end(), (int)op.a) - R.begin());
          g.mask |= (uint8_t)(1u << j);
          g.slot[j] = op.slot[0];
        }
      }
      if (g.mask) {
        // idle positions get the identity: the kernel runs all four as one straight line
        for (int j = 0; j < (int)kRegBits; ++j)
          if (!((g.mask >> j) & 1)) g.slot[j] = (uint16_t)identity_slot;
        out.push_back(g);
      }
      // sign diagonals: accumulated, then applied once by a DOP_SFLIP
      bool any_sign = false;
      for (int i : wave)
        if (ps.ops[i].type == DOP_DSIGN) {
          out.push_back(ps.ops[i]);
          any_sign = true;
        }
      if (any_sign) {
        DOp f{};
        f.type = DOP_SFLIP;
        out.push_back(f);
      }
      for (int i : wave)
        if (ps.ops[i].type != DOP_M1 && ps.ops[i].type != DOP_DSIGN) out.push_back(ps.ops[i]);
      for (int i : wave) {
        done[i] = 1;
        ++ndone;
      }
    }
    if (ndone == nops) break;
    std::vector<int> nr;
    auto try_add = [&](const DOp& op) {
      int b[2];
      int nb = local_bits(op, b);
      int add = 0;
      for (int x = 0; x < nb; ++x)
        if (std::find(nr.begin(), nr.end(), b[x]) == nr.end()) ++add;
      if ((int)nr.size() + add > (int)kRegBits) return;
      for (int x = 0; x < nb; ++x)
        if (std::find(nr.begin(), nr.end(), b[x]) == nr.end()) nr.push_back(b[x]);
    };
    for (int i = 0; i < nops && (int)nr.size() < (int)kRegBits; ++i)
      if (!done[i] && ready(i)) try_add(ps.ops[i]);
    for (int i = 0; i < nops && (int)nr.size() < (int)kRegBits; ++i)
      if (!done[i]) try_add(ps.ops[i]);
    for (int j = k - 1; j >= 0 && (int)nr.size() < (int)kRegBits; --j)
      if (std::find(nr.begin(), nr.end(), j) == nr.end()) nr.push_back(j);
    std::sort(nr.begin(), nr.end());
    if (nr == R) {
      force_wave = true;
      continue;
    }
    force_wave = false;
    out.push_back(phase_op(nr));
    R = nr;
  }
  if (R != R_io) out.push_back(phase_op(R_io));
  ps.ops.swap(out);
}

// Tile-pass schedule of a step list.  `init_zero`: the first pass starts from
// |0...0>; `phases`: order the passes for the register kernel.
static ptsbe_status schedule(Plan& plan, const std::vector<Step>& steps, std::vector<Pass>& passes,
                             std::vector<ExecStep>& exec, std::vector<std::vector<std::pair<int, int>>>& site_slots,
                             bool init_zero, bool phases, int tile_bits, bool search) {
  const int n = plan.n;
  const int k = std::min(n, tile_bits);
  // The lowest qubits are always in the tile (runs of >= 128 contiguous bytes),
  // leaving at least two free tile bits so that any 2-qubit operation fits.
  const int contiguous = std::max(0, std::min(k - 2, plan.precision == PTSBE_C64 ? 4 : 3));
  std::vector<int> rem(steps.size());
  for (size_t i = 0; i < rem.size(); ++i) rem[i] = (int)i;
  std::vector<char> measured(steps.size(), 0);
  bool first = true;
  int guard = 0;
  while (!rem.empty()) {
    if (++guard > 1000000) return fail(PTSBE_E_ARG, "scheduler made no progress");
    // greedy tile choice + take, in circuit order, from an initial tile set
    std::vector<char> inQ;
    int qcount = 0;
    std::vector<int> taken, keep;
    auto take_with = [&](const std::vector<char>& init, const std::vector<int>* from = nullptr) {
      inQ = init;
      qcount = 0;
      for (int q = 0; q < n; ++q) qcount += inQ[q];
      std::vector<char> blocked(n, 0);
      taken.clear();
      keep.clear();
      // A state-dependent channel not yet decided (forward) or restored (reverse
      // sweep) is a wall: nothing after it runs before it, so that the state at
      // its decision is the state at its place in the circuit (the checkpoint
      // the reverse sweep restores).
      bool wall = false;
      for (int si : from ? *from : rem) {
        const Step& st = steps[si];
        bool blk = wall;
        for (int j = 0; j < st.nq; ++j) blk = blk || blocked[st.q[j]];
        if (st.kind == ST_GCH && !measured[si]) wall = true;
        bool can = false;
        if (!blk) {
          if ((st.kind == ST_MR || st.kind == ST_GCH) && !measured[si]) {
            can = false;
          } else if (st.diag && st.kind != ST_MR) {
            can = true;
          } else {
            int nnew = 0;
            for (int j = 0; j < st.nq; ++j) nnew += inQ[st.q[j]] ? 0 : 1;
            if (qcount + nnew <= k) {
              for (int j = 0; j < st.nq; ++j)
                if (!inQ[st.q[j]]) {
                  inQ[st.q[j]] = 1;
                  ++qcount;
                }
              can = true;
            }
          }
        }
        if (can) {
          taken.push_back(si);
        } else {
          for (int j = 0; j < st.nq; ++j) blocked[st.q[j]] = 1;
          keep.push_back(si);
        }
      }
    };
    auto score = [&]() {
      int c = 0;
      for (int si : taken) c += steps[si].diag ? 0 : 1;
      return c;
    };
    std::vector<char> base(n, 0);
    for (int q = 0; q < contiguous; ++q) base[q] = 1;
    take_with(base);
    if (search && !taken.empty() && n > k) {
      // Tile search: among the greedy tile and every window of consecutive
      // qubits beside the contiguous ones (as wide as the tile's free part, or
      // two qubits narrower with the scan filling the rest), the tile whose
      // greedy take, plus
      // the best such take of the pass after it, runs the most non-diagonal
      // operations (on brick-like circuits a window follows a light cone
      // through many layers, where circuit order stops at the first layer's
      // boundary; looking one pass ahead avoids windows that strand the rest).
      const int free = k - contiguous;
      std::vector<std::vector<char>> cands{base};
      for (int sz : {free, free - 2})  // a window short of the tile leaves the scan two qubits
        for (int w = contiguous; sz >= 2 && w + sz <= n; ++w) {
          std::vector<char> init = base;
          for (int q = w; q < w + sz; ++q) init[q] = 1;
          cands.push_back(init);
        }
      int best = -1;
      std::vector<char> best_init = base;
      for (const auto& init : cands) {
        take_with(init);
        int sc = score();
        const std::vector<int> rest = keep;
        int next = 0;
        for (const auto& i2 : cands) {
          take_with(i2, &rest);
          next = std::max(next, score());
        }
        sc += next;
        if (sc > best) {
          best = sc;
          best_init = init;
        }
      }
      take_with(best_init);
    }
    if (taken.empty() && steps[rem[0]].kind == ST_GCH && steps[rem[0]].dagger) {
      // reverse sweep at a state-dependent channel: restore the state
      // checkpointed at its decision, apply its adjoint to lambda alone
      const Step& st = steps[rem[0]];
      ExecStep ex;
      for (int j = 0; j < st.nq; ++j) ex.mr_qubits.push_back(st.q[j]);
      ex.mr_index.push_back(st.mr);
      ex.wall = true;
      ex.restore = st.gidx;
      ex.dense = st.dense;
      exec.push_back(ex);
      rem.erase(rem.begin());
      first = false;
      continue;
    }
    if (taken.empty() && steps[rem[0]].kind == ST_GCH && steps[rem[0]].dense) {
      // a dense state-dependent channel at the front (everything before it has
      // run): its own step reduces the density matrix of its qubits, decides
      // and applies the chosen operator
      const Step& st = steps[rem[0]];
      if (first) {
        Pass p;
        p.k = k;
        for (int q = 0; q < n; ++q) (q < k ? p.tq : p.oq).push_back(q);
        p.flags = PASS_INIT_ZERO;
        passes.push_back(p);
        ExecStep e0;
        e0.pass = (int)passes.size() - 1;
        exec.push_back(e0);
        first = false;
      }
      ExecStep ex;
      for (int j = 0; j < st.nq; ++j) ex.mr_qubits.push_back(st.q[j]);
      ex.mr_index.push_back(st.mr);
      ex.wall = true;
      ex.dense = true;
      exec.push_back(ex);
      rem.erase(rem.begin());
      continue;
    }
    if (taken.empty()) {
      // every frontier operation is an undecided record entry: measure-resets are
      // decided together (their outcomes are deterministic, so they do not
      // change each other's marginals); a state-dependent channel only alone
      // among channels and only once every step before it is an entry decided
      // in this same step, so that its probabilities come from the state at its
      // place in the circuit
      ExecStep ex;
      std::vector<char> blk(n, 0);
      bool channel_pending = false, channel_taken = false, others_before = false;
      for (int si : rem) {
        const Step& st = steps[si];
        bool b = false;
        for (int j = 0; j < st.nq; ++j) b = b || blk[st.q[j]];
        const bool mr_ok = st.kind == ST_MR;
        const bool ch_ok = st.kind == ST_GCH && !st.dense && !channel_pending && !channel_taken && !others_before;
        if (!b && (mr_ok || ch_ok) && !measured[si]) {
          ex.mr_qubits.push_back(st.q[0]);
          ex.mr_index.push_back(st.mr);
          measured[si] = 1;
          channel_taken = channel_taken || st.kind == ST_GCH;
          ex.wall = ex.wall || st.kind == ST_GCH;
        } else {
          others_before = true;
        }
        if (st.kind == ST_GCH) channel_pending = true;
        for (int j = 0; j < st.nq; ++j) blk[st.q[j]] = 1;
      }
      if (ex.mr_qubits.empty()) return fail(PTSBE_E_UNSUPPORTED, "an operation does not fit in a tile");
      if (first) {
        // the state must exist before it is measured
        Pass p;
        p.k = k;
        for (int q = 0; q < n; ++q) (q < k ? p.tq : p.oq).push_back(q);
        p.flags = PASS_INIT_ZERO;
        passes.push_back(p);
        ExecStep e0;
        e0.pass = (int)passes.size() - 1;
        exec.push_back(e0);
        first = false;
      }
      exec.push_back(ex);
      continue;
    }
    for (int q = 0; q < n && qcount < k; ++q)
      if (!inQ[q]) {
        inQ[q] = 1;
        ++qcount;
      }
    Pass p;
    p.k = k;
    for (int q = 0; q < n; ++q) (inQ[q] ? p.tq : p.oq).push_back(q);
    if (first && init_zero) p.flags = PASS_INIT_ZERO;
    first = false;
    passes.push_back(p);
    Pass& ps = passes.back();
    Fuser fz(plan, steps, ps);
    for (int si : taken) fz.take(si);
    fz.finish();
    lower_signs(steps, ps);
    if (phases) schedule_phases(ps, plan.min_fill);
    ExecStep e;
    e.pass = (int)passes.size() - 1;
    exec.push_back(e);
    rem.swap(keep);
  }
  if (first) {
    Pass p;
    p.k = k;
    for (int q = 0; q < n; ++q) (q < k ? p.tq : p.oq).push_back(q);
    p.flags = init_zero ? PASS_INIT_ZERO : 0u;
    passes.push_back(p);
    ExecStep e;
    e.pass = 0;
    exec.push_back(e);
  }
  // site -> slots
  site_slots.assign(plan.sites.size(), {});
  for (size_t p = 0; p < passes.size(); ++p)
    for (size_t s = 0; s < passes[p].slots.size(); ++s)
      for (int site : passes[p].slots[s].sites) site_slots[site].push_back({(int)p, (int)s});
  for (auto& ps : passes)
    if (ps.slots.size() > 4096) return fail(PTSBE_E_UNSUPPORTED, "too many fused slots in one pass");
  return PTSBE_OK;
}

// The greedy schedule, or the tile-searched one where it needs at least 10 %
// fewer passes: a searched tile takes more operations, and on circuits where
// it saves only a pass or two (the surface code: 17 against 18) its heavier
// passes measured slower than the greedy ones.
static ptsbe_status schedule_best(Plan& plan, const std::vector<Step>& steps, std::vector<Pass>& passes,
                                  std::vector<ExecStep>& exec,
                                  std::vector<std::vector<std::pair<int, int>>>& site_slots, bool init_zero,
                                  bool phases, int tile_bits) {
  ptsbe_status st = schedule(plan, steps, passes, exec, site_slots, init_zero, phases, tile_bits, false);
  if (st != PTSBE_OK || !plan.tile_search) return st;
  std::vector<Pass> sp;
  std::vector<ExecStep> se;
  std::vector<std::vector<std::pair<int, int>>> ss;
  if (schedule(plan, steps, sp, se, ss, init_zero, phases, tile_bits, true) != PTSBE_OK) return PTSBE_OK;
  if (sp.size() * 10 <= passes.size() * 9) {
    passes.swap(sp);
    exec.swap(se);
    site_slots.swap(ss);
  }
  return PTSBE_OK;
}

// ------------------------------------------------------------ phase frames

namespace {

enum FrameEventKind { FE_M1, FE_M2, FE_DIAG, FE_BREAK };

struct FrameEvent {
  int kind, pass, slot, j;  // j: matrix qubit of an M2 slot
};

// Calls f(q, event) for every event of qubit q's chain, in program order: a
// 2x2 or 4x4 slot, a diagonal slot (D1), or a break (measure-reset, gradient
// dot, measurement step, end of program).  Diagonal ops that the tables do not
// hold as slots (signs, D2) commute with any pending diagonal and are skipped.
template <class F>
void walk_frames(int n, const std::vector<Pass>& passes, const std::vector<ExecStep>& exec, F&& f) {
  for (const ExecStep& ex : exec) {
    if (ex.pass < 0) {
      if (ex.wall)
        for (int q = 0; q < n; ++q) f(q, FrameEvent{FE_BREAK, -1, -1, 0});
      else
        for (int q : ex.mr_qubits) f(q, FrameEvent{FE_BREAK, -1, -1, 0});
      continue;
    }
    const Pass& ps = passes[ex.pass];
    for (const DOp& op : ps.ops) {
      switch (op.type) {
        case DOP_M1G:
          for (int j = 0; j < 4; ++j)
            if ((op.mask >> j) & 1) f(ps.slots[op.slot[j]].q[0], FrameEvent{FE_M1, ex.pass, op.slot[j], 0});
          break;
        case DOP_M1: f(ps.slots[op.slot[0]].q[0], FrameEvent{FE_M1, ex.pass, op.slot[0], 0}); break;
        case DOP_M2:
          f(ps.slots[op.slot[0]].q[0], FrameEvent{FE_M2, ex.pass, op.slot[0], 0});
          f(ps.slots[op.slot[0]].q[1], FrameEvent{FE_M2, ex.pass, op.slot[0], 1});
          break;
        case DOP_D1: f(ps.slots[op.slot[0]].q[0], FrameEvent{FE_DIAG, ex.pass, op.slot[0], 0}); break;
        case DOP_MR:
        case DOP_KR:
        case DOP_DOT: f(ps.tq[op.a], FrameEvent{FE_BREAK, ex.pass, -1, 0}); break;
        default: break;
      }
    }
  }
  for (int q = 0; q < n; ++q) f(q, FrameEvent{FE_BREAK, -1, -1, 0});
}

// Roles: a 2x2 slot runs with a real diagonal when the next non-diagonal event
// of its qubit is another matrix (which takes the pending diagonal in); under
// the same condition a slot that is a unitary diagonal for every choice of its
// sites (projections excluded) is merged into the pending diagonal, or, when
// noise sites can override it, keeps only the override.
void assign_frames(int n, const std::vector<Step>& steps, std::vector<Pass>& passes,
                   const std::vector<ExecStep>& exec) {
  std::vector<std::vector<FrameEvent>> chain(n);
  walk_frames(n, passes, exec, [&](int q, const FrameEvent& e) { chain[q].push_back(e); });
  auto unitary_diag = [&](const Slot& s) {
    for (const Part& pt : s.parts)
      if (!steps[pt.step].diag || steps[pt.step].kind == ST_P0) return false;
    return true;
  };
  for (int q = 0; q < n; ++q) {
    const auto& c = chain[q];
    for (size_t i = 0; i < c.size(); ++i) {
      if (c[i].kind != FE_M1 && c[i].kind != FE_DIAG && c[i].kind != FE_M2) continue;
      size_t j = i + 1;
      while (j < c.size() && c[j].kind == FE_DIAG) ++j;
      const bool absorbed = j < c.size() && (c[j].kind == FE_M1 || c[j].kind == FE_M2);
      Slot& s = passes[c[i].pass].slots[c[i].slot];
      if (c[i].kind == FE_M2) {
        s.m2_next[c[i].j] = absorbed;
        continue;
      }
      s.frame = FRAME_NONE;
      if (!absorbed) continue;
      if (unitary_diag(s)) s.frame = s.sites.empty() ? FRAME_ABSORB : (c[i].kind == FE_M1 ? FRAME_OVERRIDE_ONLY
                                                                                          : FRAME_NONE);
      else if (c[i].kind == FE_M1) s.frame = FRAME_REAL_DIAG;
    }
  }
}

// Fixed 2x2 slots (no parameter; both diagonal entries of magnitude >= 1e-2)
// of real-diagonal role hand their whole diagonal, magnitude included, to the
// pending frame instead of its phase alone: the kernels then apply them as
// x_r + c x_o, 4 FMAs per amplitude instead of 6.  The pending magnitudes
// along a qubit's chain stay within [1e-4, 1e4]; a slot that would leave them
// keeps the real diagonal (and resets them).
void unit_frames(Plan& P) {
  std::vector<std::array<double, 2>> mag(P.n, {1.0, 1.0});
  const std::map<int, int> none;
  walk_frames(P.n, P.passes, P.exec, [&](int q, const FrameEvent& e) {
    if (e.kind == FE_BREAK) {
      mag[q] = {1.0, 1.0};
      return;
    }
    Slot& s = P.passes[e.pass].slots[e.slot];
    auto in_range = [](double m) { return m >= 1e-4 && m <= 1e4; };
    if (e.kind == FE_M2) {
      // A fixed 4x4 both of whose qubits go on to another matrix takes the
      // pending diagonals in and leaves d_a (x) d_b pending, chosen (d_a0 = 1)
      // so that rows 0..2 of the stored matrix have a unit diagonal.  Decided
      // at the slot's second qubit, when both incoming magnitudes are known.
      if (e.j == 0) return;
      const int qa = s.q[0], qb = s.q[1];
      if (!s.uses_params && s.m2_next[0] && s.m2_next[1]) {
        const Mat M = slot_matrix(P, P.steps, s, nullptr, none);
        double d[3];
        for (int i = 0; i < 3; ++i) d[i] = std::abs(M[i * 5]) * mag[qa][i & 1] * mag[qb][i >> 1];
        bool ok = true;
        for (int i = 0; i < 3; ++i) ok = ok && std::abs(M[i * 5]) >= 1e-2;
        if (ok && in_range(d[1] / d[0]) && in_range(d[0]) && in_range(d[2])) {
          s.frame = FRAME_UNIT4;
          mag[qa] = {1.0, d[1] / d[0]};
          mag[qb] = {d[0], d[2]};
          return;
        }
      }
      mag[qa] = {1.0, 1.0};
      mag[qb] = {1.0, 1.0};
      return;
    }
    if (e.kind == FE_M1 && s.frame == FRAME_NONE) {  // takes the pending diagonal in
      mag[q] = {1.0, 1.0};
      return;
    }
    if (e.kind != FE_M1 || s.frame != FRAME_REAL_DIAG) return;  // unitary diagonals keep the magnitude
    if (!s.uses_params) {
      const Mat M = slot_matrix(P, P.steps, s, nullptr, none);
      const double a0 = std::abs(M[0]), a1 = std::abs(M[3]);
      const double m0 = mag[q][0] * a0, m1 = mag[q][1] * a1;
      if (a0 >= 1e-2 && a1 >= 1e-2 && in_range(m0) && in_range(m1)) {
        s.frame = FRAME_UNIT_DIAG;
        mag[q] = {m0, m1};
        return;
      }
    }
    mag[q] = {1.0, 1.0};
  });
}

cd unit_phase(cd z) {
  const double a = std::abs(z);
  return a > 0 ? z / a : cd(1, 0);
}

}  // namespace

std::vector<std::vector<SlotFrame>> slot_frames(int n, const std::vector<Pass>& passes,
                                                const std::vector<ExecStep>& exec,
                                                const std::vector<std::vector<Mat>>& defaults) {
  std::vector<std::vector<SlotFrame>> fr(passes.size());
  for (size_t p = 0; p < passes.size(); ++p) fr[p].resize(passes[p].slots.size());
  std::vector<std::array<cd, 2>> pend(n, {cd(1, 0), cd(1, 0)});
  walk_frames(n, passes, exec, [&](int q, const FrameEvent& e) {
    if (e.kind == FE_BREAK) return;  // every chain is flushed before a break (assign_frames)
    const Slot& s = passes[e.pass].slots[e.slot];
    SlotFrame& f = fr[e.pass][e.slot];

    if (e.kind == FE_M2 || (e.kind == FE_M1 && s.frame == FRAME_NONE)) {
      f.in[e.j][0] = pend[q][0];
      f.in[e.j][1] = pend[q][1];
      pend[q] = {cd(1, 0), cd(1, 0)};
      if (e.kind == FE_M2 && s.frame == FRAME_UNIT4 && e.j == 1) {
        // diagonal of M' = M (in_a (x) in_b); out_a = (1, M'11 / M'00), out_b = (M'00, M'22)
        const Mat& M = defaults[e.pass][e.slot];
        const cd m0 = M[0] * f.in[0][0] * f.in[1][0], m1 = M[5] * f.in[0][1] * f.in[1][0],
                 m2 = M[10] * f.in[0][0] * f.in[1][1];
        f.out[0] = cd(1, 0);
        f.out[1] = m1 / m0;
        f.out2[0] = m0;
        f.out2[1] = m2;
        pend[s.q[0]] = {f.out[0], f.out[1]};
        pend[s.q[1]] = {f.out2[0], f.out2[1]};
      }
    } else if (e.kind == FE_M1 && s.frame != FRAME_ABSORB) {
      f.in[0][0] = pend[q][0];
      f.in[0][1] = pend[q][1];
      const Mat& M = defaults[e.pass][e.slot];
      // a real-diagonal slot leaves the phase pending and keeps the magnitude;
      // a unit-diagonal one (and a skipped unitary diagonal) leaves it all
      const bool whole = s.frame == FRAME_UNIT_DIAG || s.frame == FRAME_OVERRIDE_ONLY;
      f.out[0] = whole ? M[0] * pend[q][0] : unit_phase(M[0] * pend[q][0]);
      f.out[1] = whole ? M[3] * pend[q][1] : unit_phase(M[3] * pend[q][1]);
      pend[q] = {f.out[0], f.out[1]};
    } else if (s.frame == FRAME_ABSORB) {
      const Mat& M = defaults[e.pass][e.slot];  // unit-modulus entries: the magnitude passes through
      pend[q] = {pend[q][0] * M[0], pend[q][1] * M[3]};
    }
  });
  return fr;
}

Mat frame_matrix(const Slot& s, const SlotFrame& f, const Mat& M) {
  Mat V = M;
  if (s.frame == FRAME_ABSORB) {
    V = mat_identity(2);
  } else if (s.type == DOP_M1) {
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) V[r * 2 + c] *= f.in[0][c];
    if (s.frame == FRAME_REAL_DIAG || s.frame == FRAME_OVERRIDE_ONLY || s.frame == FRAME_UNIT_DIAG) {
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) V[r * 2 + c] /= f.out[r];
      // the default matrix now has a real (or unit) diagonal, up to rounding,
      // which the kernels' real- and unit-diagonal forms drop; an override's is
      // general
    }
  } else if (s.type == DOP_M2) {
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) V[r * 4 + c] *= f.in[0][c & 1] * f.in[1][c >> 1];
    if (s.frame == FRAME_UNIT4)  // rows 0..2 of the default get a unit diagonal
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) V[r * 4 + c] /= f.out[r & 1] * f.out2[r >> 1];
  }
  return V;
}

ptsbe_status build_plan(const ptsbe_circuit* c, const ptsbe_noise_model* nm, const ptsbe_plan_opts* o,
                        std::shared_ptr<Plan>* out) {
  if (!c || !out) return fail(PTSBE_E_ARG, "null circuit or output handle");
  if (c->n_qubits < 1 || c->n_qubits > (uint32_t)kMaxQubits)
    return fail(c->n_qubits > (uint32_t)kMaxQubits ? PTSBE_E_UNSUPPORTED : PTSBE_E_ARG,
                "n_qubits must be in 1..35");
  if (c->n_ops && !c->ops) return fail(PTSBE_E_ARG, "null op array");
  auto plan = std::make_shared<Plan>();
  Plan& P = *plan;
  P.n = (int)c->n_qubits;
  P.precision = o ? (int)o->precision : PTSBE_C64;
  if (P.precision != PTSBE_C64 && P.precision != PTSBE_C128) return fail(PTSBE_E_ARG, "bad precision");
  int tb = (P.precision == PTSBE_C64) ? 12 : 11;
  if (o && o->tile_qubits) {
    if (o->tile_qubits < 4 || o->tile_qubits > 13)
      return fail(PTSBE_E_ARG, "tile_qubits must be in 4..13");
    tb = (int)o->tile_qubits;
    if (P.precision == PTSBE_C128 && tb > 12) return fail(PTSBE_E_ARG, "tile_qubits <= 12 for complex128");
    // 13-qubit tiles (512 threads, 64 KiB of LDS) exist only as compiled passes
    if (tb > 12 && (o->flags & PTSBE_PLAN_NO_COMPILE))
      return fail(PTSBE_E_ARG, "tile_qubits 13 needs the compiled passes (no PTSBE_PLAN_NO_COMPILE)");
  }
  P.tile_bits = tb;
  // flags bits 0..2: phase-scheduler fill threshold (0 = default 2)
  if (o && (o->flags & 7u)) P.min_fill = (int)(o->flags & 7u);
  P.use_jit = !(o && (o->flags & PTSBE_PLAN_NO_COMPILE));
  P.half_tile_lds = o && (o->flags & PTSBE_PLAN_HALF_TILE_LDS);
  P.waves = o ? (int)((o->flags >> PTSBE_PLAN_WAVES_SHIFT) & 15u) : 0;
  P.pair_fusion = !(o && (o->flags & PTSBE_PLAN_NO_PAIR_FUSION));
  if (o && (o->flags & PTSBE_PLAN_NO_SWIZZLE) && (o->flags & PTSBE_PLAN_SWIZZLE))
    return fail(PTSBE_E_ARG, "PTSBE_PLAN_SWIZZLE and PTSBE_PLAN_NO_SWIZZLE together");
  P.swizzle = (o && (o->flags & PTSBE_PLAN_NO_SWIZZLE))  ? false
              : (o && (o->flags & PTSBE_PLAN_SWIZZLE)) ? P.n > 12
                                                         : P.n >= (int)PTSBE_SWIZZLE_MIN_QUBITS;
  P.nontemporal = o && (o->flags & PTSBE_PLAN_NONTEMPORAL);
  P.tiles_per_block = (o && (o->flags & PTSBE_PLAN_TWO_TILES)) ? 2 : 1;
  P.tile_search = !(o && (o->flags & PTSBE_PLAN_NO_TILE_SEARCH));
  if (P.waves > 8) return fail(PTSBE_E_ARG, "waves per SIMD must be 0 (default) or 1..8");
  P.jit = std::make_shared<JitProgram>();
  // channels
  uint32_t n_ch = nm ? nm->n_channels : 0;
  if (n_ch && !nm->channels) return fail(PTSBE_E_ARG, "null channel array");
  for (uint32_t i = 0; i < n_ch; ++i) {
    Channel ch;
    ptsbe_status st = analyse_channel(nm->channels[i], (int)i, &ch, o && (o->flags & PTSBE_PLAN_TWIRL));
    if (st != PTSBE_OK) return st;
    P.channels.push_back(std::move(ch));
  }
  uint32_t n_rules = nm ? nm->n_rules : 0;
  if (n_rules && !nm->rules) return fail(PTSBE_E_ARG, "null rule array");
  for (uint32_t r = 0; r < n_rules; ++r) {
    const ptsbe_attach& a = nm->rules[r];
    if (a.channel >= n_ch) return fail(PTSBE_E_ARG, "rule " + std::to_string(r) + ": bad channel index");
    if (a.when > PTSBE_ATTACH_BEFORE_READOUT) return fail(PTSBE_E_ARG, "rule " + std::to_string(r) + ": bad kind");
    if (a.when != PTSBE_ATTACH_AFTER_TAG && P.channels[a.channel].nq != 1)
      return fail(PTSBE_E_ARG, "rule " + std::to_string(r) + ": measurement/readout channels act on one qubit");
    if (a.when == PTSBE_ATTACH_BEFORE_READOUT && P.n < 64 && (a.qmask >> P.n))
      return fail(PTSBE_E_ARG, "rule " + std::to_string(r) + ": readout mask names a qubit >= n");
  }
  auto add_site = [&](int ch, int nq, const int* q, uint32_t op_index, uint32_t tag,
                      uint32_t origin) -> ptsbe_status {
    if (P.channels[ch].nq != nq) return fail(PTSBE_E_ARG, "channel arity does not match the site's qubits");
    if (P.channels[ch].general) {
      // not pre-sampled: a record entry decided on the device (like a measure-reset)
      Step st;
      st.kind = ST_GCH;
      st.nq = nq;
      for (int j = 0; j < nq; ++j) st.q[j] = q[j];
      st.dense = P.channels[ch].dense;
      st.chan = ch;
      st.gidx = P.n_general++;
      st.mr = P.n_measure++;
      P.steps.push_back(st);
      return PTSBE_OK;
    }
    Site s;
    s.channel = ch;
    s.nq = nq;
    s.q[0] = q[0];
    s.q[1] = nq > 1 ? q[1] : -1;
    s.step = (int)P.steps.size();
    s.op = op_index;
    s.tag = tag;
    s.origin = origin;
    P.sites.push_back(s);
    Step st;
    st.kind = ST_SITE;
    st.nq = nq;
    for (int j = 0; j < nq; ++j) st.q[j] = q[j];
    st.site = (int)P.sites.size() - 1;
    st.diag = P.channels[ch].all_diag;
    P.steps.push_back(st);
    return PTSBE_OK;
  };
  int max_param = -1;
  for (uint32_t i = 0; i < c->n_ops; ++i) {
    const ptsbe_op& op = c->ops[i];
    std::string where = "op " + std::to_string(i) + ": ";
    if (op.nq < 1 || op.nq > 4) return fail(PTSBE_E_ARG, where + "nq must be 1..4");
    int q[4];
    for (uint32_t j = 0; j < op.nq; ++j) {
      if (op.q[j] >= (uint32_t)P.n) return fail(PTSBE_E_ARG, where + "qubit out of range");
      q[j] = (int)op.q[j];
      for (uint32_t l = 0; l < j; ++l)
        if (op.q[l] == op.q[j]) return fail(PTSBE_E_ARG, where + "repeated qubit");
    }
    if (op.kind == PTSBE_OP_GATE) {
      if (!op.mat) return fail(PTSBE_E_ARG, where + "null gate matrix");
      if (op.nq > 2) return fail(PTSBE_E_UNSUPPORTED, where + "gates on more than 2 qubits are not supported");
      Step st;
      st.kind = ST_GATE;
      st.nq = (int)op.nq;
      for (int j = 0; j < st.nq; ++j) st.q[j] = q[j];
      st.mat = read_mat(op.mat, 1 << op.nq);
      for (auto& x : st.mat)
        if (!std::isfinite(x.real()) || !std::isfinite(x.imag())) return fail(PTSBE_E_ARG, where + "non-finite matrix");
      st.diag = mat_is_diag(st.mat, 1 << op.nq);
      P.steps.push_back(st);
    } else if (op.kind == PTSBE_OP_PARAM) {
      if (op.nq != 1) return fail(PTSBE_E_ARG, where + "parametrised gates act on one qubit");
      if (op.gen < PTSBE_GEN_X || op.gen > PTSBE_GEN_Z) return fail(PTSBE_E_ARG, where + "bad generator");
      if (op.index < 0 || op.index > 1000000) return fail(PTSBE_E_ARG, where + "bad parameter index");
      Step st;
      st.kind = ST_PARAM;
      st.nq = 1;
      st.q[0] = q[0];
      st.param = op.index;
      st.gen = (int)op.gen;
      st.diag = op.gen == PTSBE_GEN_Z;
      max_param = std::max(max_param, op.index);
      P.steps.push_back(st);
    } else if (op.kind == PTSBE_OP_NOISE) {
      if (op.index < 0 || (uint32_t)op.index >= n_ch) return fail(PTSBE_E_ARG, where + "bad channel index");
      if (op.nq > 2) return fail(PTSBE_E_ARG, where + "noise ops act on 1 or 2 qubits");
      ptsbe_status s2 = add_site(op.index, (int)op.nq, q, i, op.tag, PTSBE_SITE_NOISE_OP);
      if (s2 != PTSBE_OK) return fail(s2, where + last_error_cstr());
      continue;
    } else if (op.kind == PTSBE_OP_MEASURE_RESET) {
      if (op.nq != 1) return fail(PTSBE_E_ARG, where + "measure-reset acts on one qubit");
      for (uint32_t r = 0; r < n_rules; ++r)
        if (nm->rules[r].when == PTSBE_ATTACH_BEFORE_MEASURE)
          add_site((int)nm->rules[r].channel, 1, q, i, op.tag, PTSBE_SITE_BEFORE_MEASURE);
      Step st;
      st.kind = ST_MR;
      st.nq = 1;
      st.q[0] = q[0];
      st.mr = P.n_measure++;
      P.steps.push_back(st);
      continue;
    } else if (op.kind == PTSBE_OP_PROJECT0) {
      if (op.nq != 1) return fail(PTSBE_E_ARG, where + "PROJECT0 acts on one qubit");
      Step st;
      st.kind = ST_P0;
      st.nq = 1;
      st.q[0] = q[0];
      st.mat = {cd(1, 0), cd(0, 0), cd(0, 0), cd(0, 0)};
      st.diag = true;
      P.steps.push_back(st);
      continue;
    } else {
      return fail(PTSBE_E_ARG, where + "unknown op kind");
    }
    for (uint32_t r = 0; r < n_rules; ++r) {
      const ptsbe_attach& a = nm->rules[r];
      if (a.when == PTSBE_ATTACH_AFTER_TAG && a.tag == op.tag) {
        ptsbe_status s2 = add_site((int)a.channel, (int)op.nq, q, i, op.tag, PTSBE_SITE_AFTER_TAG);
        if (s2 != PTSBE_OK) return fail(s2, where + "rule " + std::to_string(r) + ": " + last_error_cstr());
      }
    }
  }
  for (uint32_t r = 0; r < n_rules; ++r) {
    const ptsbe_attach& a = nm->rules[r];
    if (a.when != PTSBE_ATTACH_BEFORE_READOUT) continue;
    for (int qq = 0; qq < P.n; ++qq)
      if ((a.qmask >> qq) & 1) add_site((int)a.channel, 1, &qq, 0xffffffffu, 0u, PTSBE_SITE_BEFORE_READOUT);
  }
  if (P.n_measure > 65535) return fail(PTSBE_E_UNSUPPORTED, "too many measure-reset and state-dependent ops");
  if (P.n_general) {
    for (const Step& st : P.steps)
      if (st.kind == ST_P0)
        return fail(PTSBE_E_UNSUPPORTED, "projections together with state-dependent channels are not supported");
  }
  {
    // decision data of the record entries
    RecordInfo& R = P.rec_info;
    R.rec_chan.assign(P.n_measure, 0xffffffffu);
    R.rec_gidx.assign(P.n_measure, 0u);
    std::vector<int> chan_off(P.channels.size(), -1);
    for (const Step& st : P.steps) {
      if (st.kind != ST_GCH) continue;
      if (chan_off[st.chan] < 0) {
        const Channel& c = P.channels[st.chan];
        chan_off[st.chan] = (int)R.chan_param.size();
        R.chan_param.push_back((double)c.K);
        if (c.dense) {
          // K, d, then K_k^dagger K_k and K_k for every k (d x d row-major, re/im)
          const int d = 1 << c.nq;
          R.chan_param.push_back((double)d);
          for (const std::vector<Mat>* v : {&c.M, &c.U})
            for (int k = 0; k < c.K; ++k)
              for (int e = 0; e < d * d; ++e) {
                R.chan_param.push_back((*v)[k][e].real());
                R.chan_param.push_back((*v)[k][e].imag());
              }
        } else {
          for (int k = 0; k < c.K; ++k) R.chan_param.push_back(c.d0[k]);
          for (int k = 0; k < c.K; ++k) R.chan_param.push_back(c.d1[k]);
          for (int k = 0; k < c.K; ++k)
            for (int e = 0; e < 4; ++e) {
              R.chan_param.push_back(c.U[k][e].real());
              R.chan_param.push_back(c.U[k][e].imag());
            }
        }
      }
      R.rec_chan[st.mr] = (uint32_t)chan_off[st.chan];
      R.rec_gidx[st.mr] = (uint32_t)st.gidx;
    }
  }
  P.n_params = max_param + 1;
  P.site_off.push_back(0);
  for (auto& s : P.sites) {
    const Channel& ch = P.channels[s.channel];
    for (double p : ch.p) P.site_p.push_back(p);
    P.site_off.push_back((uint32_t)P.site_p.size());
  }
  ptsbe_status st = schedule_best(P, P.steps, P.passes, P.exec, P.site_slots, true, true, P.tile_bits);
  if (st != PTSBE_OK) return st;
  if (!(o && (o->flags & PTSBE_PLAN_NO_PHASE_FRAMES))) {
    assign_frames(P.n, P.steps, P.passes, P.exec);
    unit_frames(P);
  }
  // Reverse-sweep program of the adjoint gradient: the steps in reverse order,
  // each applied as its adjoint, with a DOT marker (Im<lambda|P|psi>) just before
  // un-applying every parametrised rotation.  Not for circuits with
  // measure-reset / projection; a state-dependent channel becomes a restore
  // step (its checkpointed state back into psi, its fixed operator's adjoint
  // on lambda), scheduled as a wall.
  bool unitary = true;
  for (const Step& s : P.steps) unitary = unitary && s.kind != ST_MR && s.kind != ST_P0;
  if (P.n_params > 0 && unitary) {
    Program& A = P.adj;
    int ndot = 0;
    for (int i = (int)P.steps.size() - 1; i >= 0; --i) {
      const Step& s = P.steps[i];
      if (s.kind == ST_PARAM) {
        Step d;
        d.kind = ST_DOT;
        d.nq = 1;
        d.q[0] = s.q[0];
        d.gen = s.gen;
        d.param = s.param;
        d.dot = ndot++;
        A.steps.push_back(d);
        A.dot_param.push_back(s.param);
        A.dot_gen.push_back(s.gen);
      }
      Step r = s;
      r.dagger = true;
      A.steps.push_back(r);
    }
    // two tiles (psi and lambda) share the LDS: one tile bit less
    st = schedule_best(P, A.steps, A.passes, A.exec, A.site_slots, false, true, std::max(4, P.tile_bits - 1));
    if (st != PTSBE_OK) return st;
    // A 2x2 slot that no record changes, made of one-qubit gates that are all
    // diagonal (Z rotations, phases), or all real (Y rotations, real fixed
    // gates), keeps that form for every parameter value: the sweep applies it
    // with half the arithmetic of a general complex matrix.
    // A 2x2 slot of noise sites only whose default (no error) is the identity
    // is applied only by the blocks whose trajectory overrides it.
    // A 4x4 slot without parameters whose default is a diagonal of +-1 (a CZ
    // and the noise sites after it) negates amplitudes unless overridden.
    for (Pass& ps : A.passes)
      for (Slot& sl : ps.slots) {
        if (sl.type == DOP_M2 && !sl.parts.empty()) {
          bool fixed = true;
          for (const Part& pt : sl.parts) fixed = fixed && A.steps[pt.step].kind != ST_PARAM;
          if (!fixed) continue;
          const Mat D = slot_matrix(P, A.steps, sl, nullptr, {});
          bool signs = true;
          uint8_t mask = 0;
          for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) {
              const cd z = D[r * 4 + c];
              if (r != c) signs = signs && z == cd(0, 0);
              else if (z == cd(-1, 0)) mask |= (uint8_t)(1u << r);
              else signs = signs && z == cd(1, 0);
            }
          if (signs) {
            sl.form = 6;
            sl.sign_mask = mask;
          }
          continue;
        }
        if (sl.type != DOP_M1 || sl.parts.empty()) continue;
        if (!sl.sites.empty()) {
          bool sites_only = true;
          for (const Part& pt : sl.parts) sites_only = sites_only && A.steps[pt.step].kind == ST_SITE;
          if (sites_only && slot_matrix(P, A.steps, sl, nullptr, {}) == mat_identity(2)) sl.form = 5;
          continue;
        }
        bool diag = true, real = true;
        for (const Part& pt : sl.parts) {
          const Step& s = A.steps[pt.step];
          if (pt.half >= 0 || pt.emb >= 0 || s.nq != 1 || (s.kind != ST_GATE && s.kind != ST_PARAM)) {
            diag = real = false;
            break;
          }
          diag = diag && s.diag;
          bool r = s.kind == ST_PARAM ? s.gen == PTSBE_GEN_Y : true;
          if (s.kind == ST_GATE)
            for (const cd& z : s.mat) r = r && z.imag() == 0.0;
          real = real && r;
        }
        sl.form = diag ? 4 : real ? 3 : 0;
      }
    P.has_adjoint = true;
  }
  *out = plan;
  return PTSBE_OK;
}

}  // namespace ptsbe
