// Pass compiler (see jit.hpp).  The generated kernel is the register-layout
// tile pass with the pass's operation list unrolled: 256 threads hold 16
// amplitudes each over 4 register bits of a 2^k-amplitude tile; 2x2 matrices
// on register bits are applied in registers, the register set is changed by
// an LDS transpose, and everything known per pass (tile qubits, which bits are
// register bits, which group positions are idle, which amplitudes a CZ-type
// sign touches, whether a block-uniform phase is pending) is resolved while
// generating, so the kernel executes only the arithmetic of its operations.
#include "jit.hpp"

#include <hip/hiprtc.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <set>
#include <sstream>
#include <thread>

#include "host.hpp"

namespace ptsbe {

namespace {

#define PTSBE_STR2(...) #__VA_ARGS__
#define PTSBE_STR(...) PTSBE_STR2(__VA_ARGS__)
const char* kArgsFields = PTSBE_STR(PTSBE_PASS_ARGS_FIELDS(V, void, void, DOverride, uint2));

// A Boolean runtime variable of the sign algebra: a thread bit of the local
// index or a tile (global) bit, as a C expression.
using Mono = std::vector<std::string>;  // product of variables, sorted; empty = 1

// LDS matrix entries of a pass: 4 per slot (the 2x2 view every slot has),
// then 16 per 4x4 slot, in slot order.
uint32_t lds_mat_entries(const Pass& ps) {
  uint32_t e = 4u * (uint32_t)ps.slots.size();
  for (const Slot& sl : ps.slots)
    if (sl.type == DOP_M2) e += 16u;
  return e;
}

struct Gen {
  std::ostringstream o;
  int k = 0, n = 0;
  bool c64 = true;
  std::vector<int> tq, oq;
  int R[4] = {0, 0, 0, 0};
  bool pending = false;      // `cs` holds a block-uniform scalar not yet applied
  bool cs_neg = false;       // the pending scalar must also be negated
  bool tile_read = false;    // the LDS tile was read since the last barrier
  bool split = false;        // register changes go through half a tile of LDS, in two rounds
  bool dual = false;         // adjoint sweep: every operation acts on psi (s*) and lambda (l*)
  std::vector<int> m2_off;   // slot -> offset of its 16 LDS entries (4x4 slots), else -1
  std::string pre = "s";     // register set the emitters write (s = psi, l = lambda)
  bool needs_full = false;   // an operation needs the whole tile in LDS
  // accumulated +-1 diagonal: amplitude r is negated where bit r of
  // XOR over monomials m of (value of m) * mask[m] is set
  std::map<Mono, uint32_t> signs;
  bool ok = true;
  std::string why;
  const uint8_t* frame = nullptr;  // FrameRole per slot
  const uint8_t* form = nullptr;   // reverse sweep: Slot::form per slot
  const uint8_t* smask = nullptr;  // reverse sweep: Slot::sign_mask per slot

  // bit of `slot` in the block's override set (wave-uniform words)
  std::string ovbit(int slot) const {
    return "(ovw" + std::to_string(slot >> 5) + " & " + std::to_string(1u << (slot & 31)) + "u)";
  }
  // branch condition of an override path: rare, laid out away from the hot code
  std::string ovcond(int slot) const { return "(__builtin_expect(" + ovbit(slot) + " != 0u, 0))"; }
  void load2x2(int slot) {
    o << "    V m0 = mats[" << 4 * slot << "], m1 = mats[" << 4 * slot + 1 << "], m2 = mats[" << 4 * slot + 2
      << "], m3 = mats[" << 4 * slot + 3 << "];\n";
  }

  void fail(const std::string& w) {
    if (ok) why = w;
    ok = false;
  }
  int reg_pos(int l) const {
    for (int j = 0; j < 4; ++j)
      if (R[j] == l) return j;
    return -1;
  }
  // thread-index bit that holds local bit l (l not a register bit)
  int thread_bit(int l) const {
    int i = 0;
    for (int p = 0; p < l; ++p)
      if (reg_pos(p) < 0) ++i;
    return i;
  }
  std::string tvar(int l) const { return "((tid >> " + std::to_string(thread_bit(l)) + ") & 1u)"; }
  static std::string gvar(int g) { return "((uint32_t)(base >> " + std::to_string(g) + ") & 1u)"; }
  // Lt: the thread's local-index part (register bits zero) for the current R
  std::string lt_expr() const {
    std::vector<int> P;
    for (int p = 0; p < k; ++p)
      if (reg_pos(p) < 0) P.push_back(p);
    std::string e;
    size_t i = 0;
    while (i < P.size()) {
      size_t j = i;
      while (j + 1 < P.size() && P[j + 1] == P[j] + 1) ++j;
      const uint32_t len = (uint32_t)(j - i + 1);
      // tid bits i..j land on local positions P[i]..P[j]
      std::string term = "((tid >> " + std::to_string(i) + ") & " + std::to_string((1u << len) - 1) + "u)";
      if (P[i] > 0) term = "(" + term + " << " + std::to_string(P[i]) + ")";
      e += (e.empty() ? "" : " | ") + term;
      i = j + 1;
    }
    return e.empty() ? "0u" : e;
  }
  uint32_t reg_const(int r) const {
    uint32_t c = 0;
    for (int j = 0; j < 4; ++j)
      if ((r >> j) & 1) c |= 1u << R[j];
    return c;
  }
  static uint32_t swz(uint32_t L) { return L ^ ((L >> 4) & 15u); }

  std::string S(int r) const { return pre + std::to_string(r); }
  std::vector<std::string> sets() const {
    if (dual) return {"s", "l"};
    return {"s"};
  }

  void barrier_before_tile_write() {
    if (tile_read) {
      o << "  __syncthreads();\n";
      tile_read = false;
    }
  }

  // ---- block-uniform scalar
  void apply_pending_to(const char* m0, const char* m1, const char* m2, const char* m3) {
    if (!pending) return;
    if (cs_neg) o << "    cs.x = -cs.x; cs.y = -cs.y;\n";
    o << "    " << m0 << " = cm(cs, " << m0 << "); " << m1 << " = cm(cs, " << m1 << "); " << m2 << " = cm(cs, "
      << m2 << "); " << m3 << " = cm(cs, " << m3 << ");\n";
    pending = false;
    cs_neg = false;
  }
  void pend(const std::string& ph) {
    if (pending) o << "  cs = cm(cs, " << ph << ");\n";
    else o << "  cs = " << ph << ";\n";
    pending = true;
  }

  // ---- 2x2 matrix on register position j: form 0 general, 1 real diagonal,
  // 2 unit diagonal, 3 real matrix, 4 diagonal matrix
  void gate_body(int j, int form) {
    for (const std::string& st : sets()) {
      pre = st;
      for (int r = 0; r < 16; ++r) {
        if ((r >> j) & 1) continue;
        const int r1 = r | (1 << j);
        if (form == 4)
          o << "    " << S(r) << " = cm(m0, " << S(r) << "); " << S(r1) << " = cm(m3, " << S(r1) << ");\n";
        else if (form == 3)
          o << "    { const V x0 = " << S(r) << ", x1 = " << S(r1) << "; " << S(r) << " = crr(m0.x, x0, m1.x, x1); "
            << S(r1) << " = crr(m2.x, x0, m3.x, x1); }\n";
        else if (form == 2)
          o << "    { const V x0 = " << S(r) << ", x1 = " << S(r1) << "; " << S(r) << " = cu(x0, m1, x1); " << S(r1)
            << " = cu(x1, m2, x0); }\n";
        else if (form == 1)
          o << "    { const V x0 = " << S(r) << ", x1 = " << S(r1) << "; " << S(r) << " = cr(m0.x, x0, m1, x1); "
            << S(r1) << " = cr(m3.x, x1, m2, x0); }\n";
        else
          o << "    { const V x0 = " << S(r) << ", x1 = " << S(r1) << "; " << S(r) << " = cf(m0, x0, m1, x1); "
            << S(r1) << " = cf(m2, x0, m3, x1); }\n";
      }
    }
    pre = "s";
  }
  // A slot stored with a real or unit diagonal (phase frame) runs the cheaper
  // form unless this block's trajectory overrides it with a general matrix;
  // the block-uniform scalar then stays pending instead of being folded in.
  void gate(int j, int slot) {
    const uint8_t role = frame ? frame[slot] : (uint8_t)FRAME_NONE;
    if (role == FRAME_ABSORB) return;  // merged into a pending phase frame
    o << "  {\n";
    load2x2(slot);
    if (role == FRAME_REAL_DIAG || role == FRAME_OVERRIDE_ONLY || role == FRAME_UNIT_DIAG) {
      o << "  if " << ovcond(slot) << " {\n";
      gate_body(j, 0);
      o << "  }";
      if (role != FRAME_OVERRIDE_ONLY) {
        o << " else {\n";
        gate_body(j, role == FRAME_UNIT_DIAG ? 2 : 1);
        o << "  }";
      }
      o << "\n  }\n";
      return;
    }
    // a pending block-uniform phase keeps a diagonal matrix diagonal, not a real one real
    const int f = form ? (int)form[slot] : 0;
    if (f == 5 && !pending) {
      // the identity unless this block's trajectory overrides the slot
      o << "  if " << ovcond(slot) << " {\n";
      gate_body(j, 0);
      o << "  }\n  }\n";
      return;
    }
    const int use = f == 4 || (f == 3 && !pending) ? f : 0;
    apply_pending_to("m0", "m1", "m2", "m3");
    gate_body(j, use);
    o << "  }\n";
  }

  // ---- signs
  void add_term(const Mono& m, uint32_t mask) {
    if (!mask) return;
    uint32_t& v = signs[m];
    v ^= mask;
  }
  // value of local bit / tile bit as (is_register, register pattern, variable)
  struct Bit {
    bool reg;
    uint32_t pat;       // register: 16-bit pattern over r
    std::string var;    // runtime variable otherwise
  };
  Bit bit_of_local(int l) const {
    const int j = reg_pos(l);
    if (j >= 0) {
      uint32_t p = 0;
      for (int r = 0; r < 16; ++r)
        if ((r >> j) & 1) p |= 1u << r;
      return {true, p, ""};
    }
    return {false, 0, tvar(l)};
  }
  void dsign(const DOp& op) {
    const Bit x = op.a == 255 ? Bit{false, 0, gvar(op.ga)} : bit_of_local(op.a);
    const bool one = op.b == 254;
    const Bit y = one ? Bit{true, 0, ""} : (op.b == 255 ? Bit{false, 0, gvar(op.gb)} : bit_of_local(op.b));
    const uint32_t mk = op.slot[0] & 15u;
    auto mkb = [&](int i) { return (mk >> i) & 1u; };
    // sign(r) = mk[x(r) + 2 y(r)] as a GF(2) polynomial in the runtime bits
    if (x.reg && y.reg) {
      uint32_t c = 0;
      for (int r = 0; r < 16; ++r)
        if (mkb(((x.pat >> r) & 1) + 2 * ((y.pat >> r) & 1))) c |= 1u << r;
      add_term({}, c);
    } else if (x.reg || y.reg) {
      const Bit& R_ = x.reg ? x : y;
      const std::string v = x.reg ? y.var : x.var;
      uint32_t a0 = 0, a1 = 0;
      for (int r = 0; r < 16; ++r) {
        const int rb = (R_.pat >> r) & 1;
        const int i0 = x.reg ? rb : 2 * rb;          // runtime bit = 0
        const int i1 = x.reg ? rb + 2 : 2 * rb + 1;  // runtime bit = 1
        if (mkb(i0)) a0 |= 1u << r;
        if (mkb(i1)) a1 |= 1u << r;
      }
      add_term({}, a0);
      add_term({v}, a0 ^ a1);
    } else {
      const uint32_t F = 0xFFFFu;
      add_term({}, mkb(0) ? F : 0u);
      add_term({x.var}, (mkb(0) ^ mkb(1)) ? F : 0u);
      add_term({y.var}, (mkb(0) ^ mkb(2)) ? F : 0u);
      Mono uv = {x.var, y.var};
      std::sort(uv.begin(), uv.end());
      if (uv[0] == uv[1]) add_term({x.var}, (mkb(0) ^ mkb(1) ^ mkb(2) ^ mkb(3)) ? F : 0u);
      else add_term(uv, (mkb(0) ^ mkb(1) ^ mkb(2) ^ mkb(3)) ? F : 0u);
    }
  }
  void flush_signs() {
    uint32_t c = 0;
    std::vector<std::pair<std::string, uint32_t>> rt;
    for (auto& kv : signs) {
      if (!kv.second) continue;
      if (kv.first.empty()) {
        c ^= kv.second;
      } else {
        std::string cond = kv.first[0];
        for (size_t i = 1; i < kv.first.size(); ++i) cond += " & " + kv.first[i];
        rt.push_back({cond, kv.second});
      }
    }
    signs.clear();
    if (c == 0xFFFFu && rt.empty()) {  // a sign common to the tile joins the scalar
      if (pending) cs_neg = !cs_neg;
      else {
        o << "  cs.x = -1; cs.y = 0;\n";
        pending = true;
      }
      return;
    }
    for (const std::string& st : sets()) {
      pre = st;
      for (int r = 0; r < 16; ++r)
        if ((c >> r) & 1) o << "  " << S(r) << ".x = -" << S(r) << ".x; " << S(r) << ".y = -" << S(r) << ".y;\n";
    }
    pre = "s";
    if (rt.empty()) return;
    uint32_t any = 0;
    o << "  {\n    uint32_t ng = 0u";
    for (auto& t : rt) {
      o << " ^ ((" << t.first << ") ? " << t.second << "u : 0u)";
      any |= t.second;
    }
    o << ";\n";
    for (const std::string& st : sets())
    for (int r = 0; r < 16; ++r) {
      pre = st;
      if (!((any >> r) & 1)) continue;
      if (c64)
        o << "    { const uint32_t sg = (ng << " << 31 - r << ") & 0x80000000u; " << S(r)
          << ".x = __uint_as_float(__float_as_uint(" << S(r) << ".x) ^ sg); " << S(r)
          << ".y = __uint_as_float(__float_as_uint(" << S(r) << ".y) ^ sg); }\n";
      else
        o << "    { const uint64_t sg = (uint64_t)((ng >> " << r << ") & 1u) << 63; " << S(r)
          << ".x = __longlong_as_double(__double_as_longlong(" << S(r) << ".x) ^ sg); " << S(r)
          << ".y = __longlong_as_double(__double_as_longlong(" << S(r) << ".y) ^ sg); }\n";
    }
    pre = "s";
    o << "  }\n";
  }

  // ---- diagonals
  void diag(const DOp& op) {
    const bool two = op.type == DOP_D2;
    if (op.a == 255 && (!two || op.b == 255)) {
      if (!two) {
        o << "  { const V* mp = mats + " << 4 * op.slot[0] << "; const V ph = " << gvar(op.ga)
          << " ? mp[3] : mp[0];\n  ";
        pend("ph");
        o << "  }\n";
      } else {
        o << "  { const uint32_t i = " << gvar(op.ga) << " + 2u * " << gvar(op.gb)
          << "; const V ph = a.pool[slot_off[" << op.slot[0] << "] + 5u * i];\n  ";
        pend("ph");
        o << "  }\n";
      }
      return;
    }
    o << "  {\n";
    if (!two) {
      o << "    const V d0 = mats[" << 4 * op.slot[0] << "], d1 = mats[" << 4 * op.slot[0] + 3
        << "], d2 = d0, d3 = d1;\n";
    } else {
      o << "    const V* mp = a.pool + slot_off[" << op.slot[0]
        << "]; const V d0 = mp[0], d1 = mp[5], d2 = mp[10], d3 = mp[15];\n";
    }
    auto bitexpr = [&](int local, int g, int r) -> std::string {
      if (local == 255) return gvar(g);
      const int j = reg_pos(local);
      if (j >= 0) return ((r >> j) & 1) ? "1u" : "0u";
      return tvar(local);
    };
    for (int r = 0; r < 16; ++r) {
      const std::string ba = bitexpr(op.a, op.ga, r);
      const std::string bb = two ? bitexpr(op.b, op.gb, r) : "0u";
      std::string e;
      auto pick = [&](const std::string& b, const std::string& lo, const std::string& hi) {
        if (b == "0u") return lo;
        if (b == "1u") return hi;
        return "(" + b + " ? " + hi + " : " + lo + ")";
      };
      const std::string lo = pick(ba, "d0", "d1"), hi = pick(ba, "d2", "d3");
      e = pick(bb, lo, hi);
      for (const std::string& st : sets()) {
        pre = st;
        o << "    " << S(r) << " = cm(" << e << ", " << S(r) << ");\n";
      }
      pre = "s";
    }
    o << "  }\n";
  }

  // ---- 4x4 matrix
  void m2(const DOp& op) {
    const int ja = reg_pos(op.a), jb = reg_pos(op.b);
    if (ja >= 0 && jb >= 0 && op.slot[0] < m2_off.size() && m2_off[op.slot[0]] >= 0) {
      // unit4: rows 0..2 of the stored default have a unit diagonal (phase
      // frame); a block whose trajectory overrides the slot runs all 4 rows
      // in full
      const bool unit4 = frame && frame[op.slot[0]] == FRAME_UNIT4;
      auto rows = [&](bool unit) {
        for (const std::string& st : sets())
        for (int r = 0; r < 16; ++r) {
          pre = st;
          if ((r >> ja) & 1 || (r >> jb) & 1) continue;
          const int i0 = r, i1 = r | (1 << ja), i2 = r | (1 << jb), i3 = r | (1 << ja) | (1 << jb);
          o << "    { const V x0 = " << S(i0) << ", x1 = " << S(i1) << ", x2 = " << S(i2) << ", x3 = " << S(i3)
            << ";\n";
          const int idx[4] = {i0, i1, i2, i3};
          for (int q = 0; q < 4; ++q) {
            o << "      " << S(idx[q]) << " = ";
            if (unit && q < 3) {
              // x_q + the other three entries of row q
              o << "cu3(x" << q;
              for (int c = 0; c < 4; ++c)
                if (c != q) o << ", M[" << 4 * q + c << "], x" << c;
              o << ");\n";
            } else {
              o << "cd4(M + " << 4 * q << ", x0, x1, x2, x3);\n";
            }
          }
          o << "    }\n";
        }
        pre = "s";
      };
      const int f = form ? (int)form[op.slot[0]] : 0;
      o << "  {\n    const V* M = mats + " << m2_off[op.slot[0]] << ";\n";
      if (f == 6) {
        // a default of +-1 on the diagonal: negations, the matrix where overridden
        o << "  if " << ovcond(op.slot[0]) << " {\n";
        rows(false);
        o << "  } else {\n";
        const uint32_t mk = smask[op.slot[0]];
        for (const std::string& st : sets()) {
          pre = st;
          for (int r = 0; r < 16; ++r) {
            if ((r >> ja) & 1 || (r >> jb) & 1) continue;
            const int idx[4] = {r, r | (1 << ja), r | (1 << jb), r | (1 << ja) | (1 << jb)};
            for (int q = 0; q < 4; ++q)
              if ((mk >> q) & 1) o << "    " << S(idx[q]) << ".x = -" << S(idx[q]) << ".x; " << S(idx[q]) << ".y = -"
                                   << S(idx[q]) << ".y;\n";
          }
        }
        pre = "s";
        o << "  }\n  }\n";
        return;
      }
      if (unit4) {
        o << "  if " << ovcond(op.slot[0]) << " {\n";
        rows(false);
        o << "  } else {\n";
        rows(true);
        o << "  }\n";
      } else {
        rows(false);
      }
      o << "  }\n";
      return;
    }
    o << "  {\n    const V* m = a.pool + slot_off[" << op.slot[0] << "];\n";
    if (ja >= 0 && jb >= 0) {
      o << "    V M[16];\n    for (int i = 0; i < 16; ++i) M[i] = m[i];\n";
      for (const std::string& st : sets())
      for (int r = 0; r < 16; ++r) {
        pre = st;
        if ((r >> ja) & 1 || (r >> jb) & 1) continue;
        const int i0 = r, i1 = r | (1 << ja), i2 = r | (1 << jb), i3 = r | (1 << ja) | (1 << jb);
        o << "    { const V x0 = " << S(i0) << ", x1 = " << S(i1) << ", x2 = " << S(i2) << ", x3 = " << S(i3) << ";\n";
        const int idx[4] = {i0, i1, i2, i3};
        for (int q = 0; q < 4; ++q)
          o << "      " << S(idx[q]) << " = cd4(M + " << 4 * q << ", x0, x1, x2, x3);\n";
        o << "    }\n";
      }
      pre = "s";
      o << "  }\n";
      return;
    }
    // through the LDS tile: any two local bits
    needs_full = true;
    o << "    const uint32_t Lt = " << lt_expr() << ", Lw = Lt ^ ((Lt >> 4) & 15u);\n";
    for (const std::string& st : sets()) {
    pre = st;
    barrier_before_tile_write();
    for (int r = 0; r < 16; ++r) o << "    tile[Lw ^ " << swz(reg_const(r)) << "u] = " << S(r) << ";\n";
    o << "    __syncthreads();\n";
    const uint32_t A = 1u << op.a, B = 1u << op.b;
    const uint32_t l1 = std::min(A, B) - 1, l2 = std::max(A, B) - 1;
    o << "    for (uint32_t qd = tid; qd < " << (1u << (k - 2)) << "u; qd += blockDim.x) {\n"
      << "      uint32_t i = ((qd & ~" << l1 << "u) << 1) | (qd & " << l1 << "u);\n"
      << "      i = ((i & ~" << l2 << "u) << 1) | (i & " << l2 << "u);\n"
      << "      const uint32_t i0 = sw(i), i1 = sw(i | " << A << "u), i2 = sw(i | " << B << "u), i3 = sw(i | "
      << (A | B) << "u);\n"
      << "      const V x0 = tile[i0], x1 = tile[i1], x2 = tile[i2], x3 = tile[i3];\n"
      << "      tile[i0] = cd4(m, x0, x1, x2, x3); tile[i1] = cd4(m + 4, x0, x1, x2, x3);\n"
      << "      tile[i2] = cd4(m + 8, x0, x1, x2, x3); tile[i3] = cd4(m + 12, x0, x1, x2, x3);\n    }\n"
      << "    __syncthreads();\n";
    for (int r = 0; r < 16; ++r) o << "    " << S(r) << " = tile[Lw ^ " << swz(reg_const(r)) << "u];\n";
    tile_read = true;
    }
    pre = "s";
    o << "  }\n";
  }

  void mr(const DOp& op) {
    const int j = reg_pos(op.a);
    if (j < 0 || dual) {
      fail("measure-reset on a non-register bit or in an adjoint sweep");
      return;
    }
    o << "  {\n    const uint64_t ri = (uint64_t)t * a.n_measure + " << op.slot[0]
      << "u;\n    const uint32_t b = a.mr_bits[ri];\n    const T sc = (T)a.mr_norm[ri];\n";
    for (int r = 0; r < 16; ++r) {
      if ((r >> j) & 1) continue;
      const int r1 = r | (1 << j);
      o << "    { V x = b ? " << S(r1) << " : " << S(r) << "; x.x *= sc; x.y *= sc; " << S(r) << " = x; " << S(r1)
        << ".x = 0; " << S(r1) << ".y = 0; }\n";
    }
    o << "  }\n";
  }

  // state-dependent channel: K_k / sqrt(p_k) on register position j, k and the
  // factor from the trajectory's record entry, K_0.. at the slot's pool offset
  void kr(const DOp& op) {
    const int j = reg_pos(op.a);
    if (j < 0 || dual) {
      fail("state-dependent channel on a non-register bit or in an adjoint sweep");
      return;
    }
    o << "  {\n    const uint64_t ri = (uint64_t)t * a.n_measure + " << op.slot[0] << "u;\n"
      << "    const T sc = (T)a.mr_norm[ri];\n"
      << "    const V* kp = a.pool + slot_off[" << op.slot[1] << "] + 4u * a.mr_bits[ri];\n"
      << "    V m0 = kp[0], m1 = kp[1], m2 = kp[2], m3 = kp[3];\n"
      << "    m0.x *= sc; m0.y *= sc; m1.x *= sc; m1.y *= sc; m2.x *= sc; m2.y *= sc; m3.x *= sc; m3.y *= sc;\n";
    apply_pending_to("m0", "m1", "m2", "m3");
    gate_body(j, 0);
    o << "  }\n";
  }

  void phase(const DOp& op) {
    if (!signs.empty()) {
      bool live = false;
      for (auto& kv : signs) live |= kv.second != 0;
      if (live) fail("signs pending across a register change");
    }
    barrier_before_tile_write();
    int nr[4] = {op.a, op.b, op.ga, op.gb};
    if (split) {
      phase_split(nr);
      return;
    }
    int oldR[4] = {R[0], R[1], R[2], R[3]};
    for (const std::string& st : sets()) {
      pre = st;
      barrier_before_tile_write();
      for (int j = 0; j < 4; ++j) R[j] = oldR[j];
      o << "  {\n    const uint32_t Lt = " << lt_expr() << ", Lw = Lt ^ ((Lt >> 4) & 15u);\n";
      for (int r = 0; r < 16; ++r) o << "    tile[Lw ^ " << swz(reg_const(r)) << "u] = " << S(r) << ";\n";
      o << "  }\n  __syncthreads();\n";
      for (int j = 0; j < 4; ++j) R[j] = nr[j];
      for (int j = 0; j < 3; ++j)
        if (!(R[j] < R[j + 1]) || R[3] >= k) fail("register bits not ascending");
      o << "  {\n    const uint32_t Lt = " << lt_expr() << ", Lw = Lt ^ ((Lt >> 4) & 15u);\n";
      for (int r = 0; r < 16; ++r) o << "    " << S(r) << " = tile[Lw ^ " << swz(reg_const(r)) << "u];\n";
      o << "  }\n";
      tile_read = true;
    }
    pre = "s";
  }

  // ---- adjoint gradient term: Im<lambda|P|psi> over this tile, P = X/Y/Z on a
  // register bit; each wavefront sums its lanes and writes one FP64 partial
  void dot(const DOp& op) {
    const int j = reg_pos(op.a);
    if (j < 0 || !dual) {
      fail("gradient term on a non-register bit");
      return;
    }
    const uint32_t d = (uint32_t)op.slot[0] | ((uint32_t)op.slot[1] << 16);
    // the thread's 8 products are summed in the state's precision, the
    // wavefront and everything above it in FP64
    o << "  {\n    T acc_t = 0;\n";
    for (int r = 0; r < 16; ++r) {
      if ((r >> j) & 1) continue;
      const int r1 = r | (1 << j);
      const std::string p0 = "s" + std::to_string(r), p1 = "s" + std::to_string(r1);
      const std::string l0 = "l" + std::to_string(r), l1 = "l" + std::to_string(r1);
      if (op.b == 3)
        o << "    acc_t += imc(" << l0 << ", " << p0 << ") - imc(" << l1 << ", " << p1 << ");\n";
      else if (op.b == 1)
        o << "    acc_t += imc(" << l0 << ", " << p1 << ") + imc(" << l1 << ", " << p0 << ");\n";
      else  // Y: (Y psi)_0 = -i psi_1, (Y psi)_1 = i psi_0
        o << "    acc_t += rec(" << l1 << ", " << p0 << ") - rec(" << l0 << ", " << p1 << ");\n";
    }
    o << "    double acc = (double)acc_t;\n";
    const uint32_t bd = 1u << (k - 4), wl = std::min<uint32_t>(64, bd);
    for (uint32_t off = 1; off < wl; off <<= 1) o << "    acc += __shfl_xor(acc, " << off << ", " << wl << ");\n";
    const uint32_t W = bd / wl;
    o << "    if ((tid & " << wl - 1 << "u) == 0u) partial[((uint64_t)t * " << (1ull << (n - k)) * W
      << "ull + tile_id * " << W << "ull + (tid / " << wl << "u)) * n_dot + " << d << "u] = acc;\n  }\n";
  }

  // local index with bit p removed
  static uint32_t compress(uint32_t L, int p) { return ((L >> (p + 1)) << p) | (L & ((1u << p) - 1u)); }
  std::string compress_expr(const std::string& L, int p) const {
    return "(((" + L + ") >> " + std::to_string(p + 1) + ") << " + std::to_string(p) + ") | ((" + L + ") & " +
           std::to_string((1u << p) - 1u) + "u)";
  }
  // One side (write: old layout, read: new layout) of a half-tile round h:
  // the amplitudes whose local bit p equals h move through tile[0 .. 2^(k-1)).
  // Reads of amplitude r go to u<r> instead of s<r> where defer[r] is set.
  void half_side(bool write, int p, int h, const bool* defer) {
    const int j = reg_pos(p);
    const std::string lt = lt_expr();
    o << "  {\n    const uint32_t Lt = " << lt << ";\n    const uint32_t Lc = " << compress_expr("Lt", p)
      << ", Lw = Lc ^ ((Lc >> 4) & 15u);\n";
    std::string indent = "    ";
    if (j < 0) {  // p is a thread bit: this thread moves all or none of its amplitudes
      o << "    if (((tid >> " << thread_bit(p) << ") & 1u) == " << h << "u) {\n";
      indent = "      ";
    }
    for (int r = 0; r < 16; ++r) {
      if (j >= 0 && ((r >> j) & 1) != h) continue;
      const uint32_t c = swz(compress(reg_const(r), p));
      if (write) o << indent << "tile[Lw ^ " << c << "u] = " << S(r) << ";\n";
      else o << indent << (defer && defer[r] ? "u" + std::to_string(r) : S(r)) << " = tile[Lw ^ " << c << "u];\n";
    }
    if (j < 0) o << "    }\n";
    o << "  }\n";
  }
  void phase_split(const int* nr) {
    int newR[4] = {nr[0], nr[1], nr[2], nr[3]};
    for (int j = 0; j < 3; ++j)
      if (!(newR[j] < newR[j + 1]) || newR[3] >= k) fail("register bits not ascending");
    // partition bit: a register bit in both layouts if any, else one in either
    int p = -1;
    for (int j = 0; j < 4 && p < 0; ++j)
      for (int i = 0; i < 4; ++i)
        if (R[j] == newR[i]) p = R[j];
    if (p < 0) p = R[3];
    int oldR[4] = {R[0], R[1], R[2], R[3]};
    const int jo = reg_pos(p);
    for (int j = 0; j < 4; ++j) R[j] = newR[j];
    const int jn = reg_pos(p);
    // a round-0 read must not overwrite a register that round 1 still writes
    bool defer[16];
    bool any = false;
    for (int r = 0; r < 16; ++r) {
      const bool read0 = jn < 0 || ((r >> jn) & 1) == 0;
      const bool write1 = jo < 0 || ((r >> jo) & 1) == 1;
      defer[r] = read0 && write1;
      any |= defer[r];
    }
    o << "  {\n";
    for (int r = 0; r < 16; ++r)
      if (defer[r]) o << "  V u" << r << ";\n";
    for (int h = 0; h < 2; ++h) {
      if (h) o << "  __syncthreads();\n";
      for (int j = 0; j < 4; ++j) R[j] = oldR[j];
      half_side(true, p, h, nullptr);
      o << "  __syncthreads();\n";
      for (int j = 0; j < 4; ++j) R[j] = newR[j];
      half_side(false, p, h, h == 0 ? defer : nullptr);
    }
    if (any) {
      std::string indent = "  ";
      if (jn < 0) {  // only the threads that read in round 0 hold deferred values
        o << "  if (((tid >> " << thread_bit(p) << ") & 1u) == 0u) {\n";
        indent = "    ";
      }
      for (int r = 0; r < 16; ++r)
        if (defer[r]) o << indent << S(r) << " = u" << r << ";\n";
      if (jn < 0) o << "  }\n";
    }
    o << "  }\n";
    tile_read = true;
  }
};

const char* kPrelude = R"(typedef __UINT8_TYPE__ uint8_t;
typedef __UINT32_TYPE__ uint32_t;
typedef __UINT64_TYPE__ uint64_t;
struct DOverride { uint32_t slot, off; };
)";

const char* kHelpers = R"(
__device__ __forceinline__ V cm(V a, V b) { V r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r; }
__device__ __forceinline__ V cf(V m0, V x0, V m1, V x1) {
  V r;
  r.x = m0.x * x0.x - m0.y * x0.y + m1.x * x1.x - m1.y * x1.y;
  r.y = m0.x * x0.y + m0.y * x0.x + m1.x * x1.y + m1.y * x1.x;
  return r;
}
// d * xd + m * xo for a real d: the diagonal entry of a phase-frame matrix
__device__ __forceinline__ V cr(T d, V xd, V m, V xo) {
  V r;
  r.x = d * xd.x + m.x * xo.x - m.y * xo.y;
  r.y = d * xd.y + m.x * xo.y + m.y * xo.x;
  return r;
}
// xd + m * xo: a row with a unit diagonal entry
__device__ __forceinline__ V cu(V xd, V m, V xo) {
  V r;
  r.x = xd.x + m.x * xo.x - m.y * xo.y;
  r.y = xd.y + m.x * xo.y + m.y * xo.x;
  return r;
}
// xd + m1 * x1 + m2 * x2 + m3 * x3: a 4x4 row with a unit diagonal entry
__device__ __forceinline__ V cu3(V xd, V m1, V x1, V m2, V x2, V m3, V x3) {
  V r;
  r.x = xd.x + m1.x * x1.x - m1.y * x1.y + m2.x * x2.x - m2.y * x2.y + m3.x * x3.x - m3.y * x3.y;
  r.y = xd.y + m1.x * x1.y + m1.y * x1.x + m2.x * x2.y + m2.y * x2.x + m3.x * x3.y + m3.y * x3.x;
  return r;
}
// one row of a 4x4 matrix: one multiply-add chain per component (1 multiply
// and 7 FMAs, against 2 + 6 + 1 add for two 2-term rows summed)
__device__ __forceinline__ V cd4(const V* m, V x0, V x1, V x2, V x3) {
  V r;
  r.x = m[0].x * x0.x - m[0].y * x0.y + m[1].x * x1.x - m[1].y * x1.y + m[2].x * x2.x - m[2].y * x2.y +
        m[3].x * x3.x - m[3].y * x3.y;
  r.y = m[0].x * x0.y + m[0].y * x0.x + m[1].x * x1.y + m[1].y * x1.x + m[2].x * x2.y + m[2].y * x2.x +
        m[3].x * x3.y + m[3].y * x3.x;
  return r;
}
__device__ __forceinline__ uint32_t sw(uint32_t L) { return L ^ ((L >> 4) & 15u); }
__device__ __forceinline__ V ldnt(const V* p) {
  V r;
  r.x = __builtin_nontemporal_load(&p->x);
  r.y = __builtin_nontemporal_load(&p->y);
  return r;
}
__device__ __forceinline__ void stnt(V* p, V v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}
)";

// helpers of the adjoint sweep's gradient terms: Im(conj(a) b) and Re(conj(a) b)
// in the state's precision
const char* kDualHelpers = R"(__device__ __forceinline__ T imc(V a, V b) { return a.x * b.y - a.y * b.x; }
__device__ __forceinline__ T rec(V a, V b) { return a.x * b.x + a.y * b.y; }
// a * x0 + b * x1 for real a, b: a row of a real 2x2 matrix
__device__ __forceinline__ V crr(T a, V x0, T b, V x1) {
  V r;
  r.x = a * x0.x + b * x1.x;
  r.y = a * x0.y + b * x1.y;
  return r;
}
)";

std::string bit_gather(const char* src, const std::vector<int>& dst_pos, int first_src_bit) {
  // sum over i of ((src >> (first + i)) & 1) << dst_pos[i], as shifted runs (64-bit)
  std::string e;
  size_t i = 0;
  while (i < dst_pos.size()) {
    size_t j = i;
    while (j + 1 < dst_pos.size() && dst_pos[j + 1] == dst_pos[j] + 1) ++j;
    const int len = (int)(j - i + 1);
    const int sb = first_src_bit + (int)i;
    std::string term = "(((uint64_t)" + std::string(src) + " >> " + std::to_string(sb) + ") & " +
                       std::to_string((1ull << len) - 1) + "ull)";
    term = "(" + term + " << " + std::to_string(dst_pos[i]) + ")";
    e += (e.empty() ? "" : " | ") + term;
    i = j + 1;
  }
  return e.empty() ? "0ull" : e;
}

}  // namespace

namespace {

std::string gen_pass(const Pass& ps, int n, int precision, const std::string& name, bool split, bool dual,
                     int waves, bool swz, bool nt, int tpb, bool* needs_full) {
  const int k = ps.k;
  if (k < (int)kMinRegTile || k > 13 || (dual && k > 12)) return "";
  if (dual && (ps.flags & PASS_INIT_ZERO)) return "";
  // The reverse sweep holds psi and lambda in registers (64 of them for the
  // amplitudes); left to itself the compiler can settle on two waves per SIMD
  // where three fit with a few spilled registers and run faster.
  if (dual && waves == 0) waves = 3;
  // two tiles per workgroup: tiles 2b and 2b + 1 of the block's state (they
  // differ in the lowest qubit outside the tile); forward passes only
  const bool two = tpb == 2 && !dual && n > k;
  Gen g;
  g.split = split && !dual;
  g.dual = dual;
  split = g.split;
  g.k = k;
  g.n = n;
  g.c64 = precision == PTSBE_C64;
  g.tq = ps.tq;
  g.oq = ps.oq;
  for (int j = 0; j < 4; ++j) g.R[j] = k - 4 + j;
  const int n_slots = (int)ps.slots.size();
  // 4x4 slots also keep all 16 entries in LDS, after the 2x2 views
  g.m2_off.assign(n_slots, -1);
  std::vector<std::pair<int, int>> m2_blocks;  // (slot, LDS offset)
  {
    int off = 4 * n_slots;
    for (int i = 0; i < n_slots; ++i)
      if (ps.slots[i].type == DOP_M2) {
        g.m2_off[i] = off;
        m2_blocks.push_back({i, off});
        off += 16;
      }
  }
  std::vector<uint8_t> frame(n_slots);
  std::set<int> ovw_words;  // words of the override bit set that hold a rewritten 2x2 slot
  for (int i = 0; i < n_slots; ++i) {
    frame[i] = ps.slots[i].frame;
    if (frame[i] == FRAME_REAL_DIAG || frame[i] == FRAME_OVERRIDE_ONLY || frame[i] == FRAME_UNIT_DIAG ||
        frame[i] == FRAME_UNIT4)
      ovw_words.insert(i >> 5);
  }
  g.frame = frame.data();
  std::vector<uint8_t> form(n_slots), smask(n_slots);
  for (int i = 0; i < n_slots; ++i) {
    form[i] = dual ? ps.slots[i].form : 0;
    smask[i] = ps.slots[i].sign_mask;
    if (form[i] == 5 || form[i] == 6) ovw_words.insert(i >> 5);
  }
  g.form = form.data();
  g.smask = smask.data();
  const int n_ovw = (n_slots + 31) / 32;
  std::ostringstream& o = g.o;
  o << kPrelude << (g.c64 ? "typedef float T;\ntypedef float2 V;\n" : "typedef double T;\ntypedef double2 V;\n")
    << "struct PassArgs { " << kArgsFields << " };\n"
    << "static_assert(sizeof(PassArgs) == " << sizeof(PassArgs<float2>) << ", \"PassArgs layout\");\n"
    << kHelpers << (dual ? kDualHelpers : "");
  o << "extern \"C\" __global__ __launch_bounds__(" << std::max(256, 1 << (k - 4)) << ") ";
  if (waves > 0) o << "__attribute__((amdgpu_waves_per_eu(" << waves << "))) ";
  o << "void " << name << "(PassArgs a"
    << (dual ? ", V* lam, double* partial, uint32_t n_dot" : "") << ") {\n"
    << "  extern __shared__ __align__(16) unsigned char smem[];\n"
    << "  V* tile = reinterpret_cast<V*>(smem);\n"
    << "  V* mats = tile + " << (split ? (1 << (k - 1)) : (1 << k)) << ";\n"
    << "  uint32_t* slot_off = reinterpret_cast<uint32_t*>(mats + " << lds_mat_entries(ps) << ");\n"
    << "  const uint32_t tid = threadIdx.x;\n"
    << "  uint32_t src = blockIdx.y, dst = blockIdx.y;\n"
    << "  if (a.route) { const uint2 e = a.route[blockIdx.y]; src = e.x; dst = e.y; }\n"
    << "  const bool carrier = a.route != nullptr && dst >= a.carrier0;\n"
    << "  const uint32_t t = carrier ? a.carrier_t : a.t0 + dst;\n";
  // The state loads come first: their latency overlaps the matrix set-up.
  // Global offsets: thread part from tid, register parts constant.
  std::vector<int> tpos(g.tq.begin(), g.tq.begin() + (k - 4));
  o << "  const uint64_t ot = " << bit_gather("tid", tpos, 0) << ";\n";
  if (two)
    o << "  const uint64_t tile_id0 = 2ull * blockIdx.x;\n"
      << "  const uint64_t base_a = " << bit_gather("tile_id0", g.oq, 0) << ";\n"
      << "  const uint64_t base_b = base_a | " << (1ull << g.oq[0]) << "ull;\n"
      << "  V cs; cs.x = 1; cs.y = 0;\n";
  else
    o << "  const uint64_t tile_id = blockIdx.x;\n"
      << "  const uint64_t base = " << bit_gather("tile_id", g.oq, 0) << ";\n"
      << "  V cs; cs.x = 1; cs.y = 0;\n";
  uint64_t og[16];
  for (int r = 0; r < 16; ++r) {
    og[r] = 0;
    for (int j = 0; j < 4; ++j)
      if ((r >> j) & 1) og[r] |= 1ull << g.tq[k - 4 + j];
  }
  // Storage positions (states swizzled, kernels.hpp): amplitude base | ot | og[r]
  // sits at px ^ og[r] ^ (f(og[r] >> 12) << 4) with px = (base | ot) ^ ((f(base >> 12)
  // ^ f(ot >> 12)) << 4), f linear; the register part is a constant.
  swz = swz && n > 12;
  std::string pos_base = "base + ot";
  // f(tile part) ^ f(thread part) of the swizzle, for the tile id in `tv`
  auto fx_of = [&](const std::string& tv) {
    std::string fx;
    for (size_t j = 0; j < g.oq.size(); ++j)
      if (g.oq[j] >= 12)
        fx += " ^ ((uint32_t)((" + tv + " >> " + std::to_string(j) + ") & 1u) * " +
              std::to_string(kSwizzle[g.oq[j] - 12]) + "u)";
    for (size_t j = 0; j < tpos.size(); ++j)
      if (tpos[j] >= 12)
        fx += " ^ (((tid >> " + std::to_string(j) + ") & 1u) * " + std::to_string(kSwizzle[tpos[j] - 12]) + "u)";
    return fx;
  };
  if (swz) {
    if (two) {
      o << "  const uint64_t px_a = (base_a + ot) ^ ((uint64_t)(0u" << fx_of("tile_id0") << ") << 4);\n"
        << "  const uint64_t px_b = (base_b + ot) ^ ((uint64_t)(0u" << fx_of("(tile_id0 + 1ull)") << ") << 4);\n";
    } else {
      o << "  const uint64_t px = (base + ot) ^ ((uint64_t)(0u" << fx_of("tile_id") << ") << 4);\n";
    }
    pos_base = "px";
    for (int r = 0; r < 16; ++r) {
      uint32_t fr = 0;
      for (int j = 0; j < 4; ++j)
        if (((r >> j) & 1) && g.tq[k - 4 + j] >= 12) fr ^= kSwizzle[g.tq[k - 4 + j] - 12];
      og[r] ^= (uint64_t)fr << 4;   // applied by XOR onto px
    }
  }
  const char* join = swz ? " ^ " : " + ";
  const bool init = (ps.flags & PASS_INIT_ZERO) != 0;
  auto emit_init = [&]() {  // |0...0> on the loop's current tile (registers declared before the loop)
    o << "  s0.x = (base == 0 && tid == 0) ? (T)1 : (T)0; s0.y = 0;\n";
    for (int r = 1; r < 16; ++r) o << "  " << g.S(r) << ".x = 0; " << g.S(r) << ".y = 0;\n";
  };
  if (two) {
    // the second tile's loads are issued with the first's; its registers
    // become the working set after the first tile is stored
    const std::string pa = swz ? "px_a" : "base_a + ot", pb = swz ? "px_b" : "base_b + ot";
    if (init) {
      o << "  V";
      for (int r = 0; r < 16; ++r) o << (r ? ", " : " ") << g.S(r);
      o << ";\n";
    } else {
      o << "  const V* sst = a.states + (uint64_t)src * a.N;\n";
      for (int h = 0; h < 2; ++h)
        for (int r = 0; r < 16; ++r) {
          const std::string at = "(" + (h ? pb : pa) + ")" + join + std::to_string(og[r]) + "ull";
          o << "  V " << (h ? "b" + std::to_string(r) : g.S(r)) << " = "
            << (nt ? "ldnt(sst + (" + at + "))" : "sst[" + at + "]") << ";\n";
        }
    }
  } else if (init) {
    o << "  V s0; s0.x = (base == 0 && tid == 0) ? (T)1 : (T)0; s0.y = 0;\n";
    for (int r = 1; r < 16; ++r) o << "  V " << g.S(r) << "; " << g.S(r) << ".x = 0; " << g.S(r) << ".y = 0;\n";
  } else {
    o << "  const V* sst = a.states + (uint64_t)src * a.N;\n";
    for (int r = 0; r < 16; ++r) {
      const std::string at = "(" + pos_base + ")" + join + std::to_string(og[r]) + "ull";
      o << "  V " << g.S(r) << " = " << (nt ? "ldnt(sst + (" + at + "))" : "sst[" + at + "]") << ";\n";
    }
    if (dual) {
      o << "  const V* lst = lam + (uint64_t)src * a.N;\n";
      for (int r = 0; r < 16; ++r) o << "  V l" << r << " = lst[(" << pos_base << ")" << join << og[r] << "ull];\n";
    }
  }
  // Matrix set-up in LDS: every block gathers the defaults (one dependent
  // pair of loads, overlapping the state loads); only a block whose trajectory
  // overrides slots of this pass patches them after a barrier.
  o << "  uint32_t* ovw = slot_off + " << n_slots << ";\n"
    << "  uint32_t ob = 0u, oe = 0u;\n"
    << "  if (!carrier) {\n"
    << "    ob = a.ov_off[(uint64_t)t * a.n_passes + a.pass];\n"
    << "    oe = a.ov_off[(uint64_t)t * a.n_passes + a.pass + 1];\n"
    << "  }\n"
    << "  for (uint32_t i = tid; i < " << n_slots << "u; i += blockDim.x) slot_off[i] = a.slot_default[i];\n"
    << "  for (uint32_t i = tid; i < " << 4 * n_slots
    << "u; i += blockDim.x) mats[i] = a.pool[a.slot_default[i >> 2] + (i & 3u)];\n";
  for (const auto& b : m2_blocks)
    o << "  for (uint32_t i = tid; i < 16u; i += blockDim.x) mats[" << b.second << "u + i] = a.pool[a.slot_default["
      << b.first << "] + i];\n";
  o << "  for (uint32_t i = tid; i < " << n_ovw << "u; i += blockDim.x) ovw[i] = 0u;\n"
    << "  __syncthreads();\n"
    << "  if (ob != oe) {\n"
    << "    for (uint32_t i = ob + tid; i < oe; i += blockDim.x) {\n"
    << "      const uint32_t sl = a.ov[i].slot, off = a.ov[i].off;\n"
    << "      slot_off[sl] = off;\n"
    << "      for (uint32_t e = 0; e < 4u; ++e) mats[4u * sl + e] = a.pool[off + e];\n";
  if (!m2_blocks.empty()) {
    o << "      switch (sl) {\n";
    for (const auto& b : m2_blocks)
      o << "        case " << b.first << "u: for (uint32_t e = 0; e < 16u; ++e) mats[" << b.second
        << "u + e] = a.pool[off + e]; break;\n";
    o << "        default: break;\n      }\n";
  }
  o
    << "      atomicOr(ovw + (sl >> 5), 1u << (sl & 31u));\n"
    << "    }\n"
    << "    __syncthreads();\n"
    << "  }\n";
  // which rewritten slots this block's trajectory overrides, as wave-uniform words
  for (int w : ovw_words)
    o << "  const uint32_t ovw" << w << " = __builtin_amdgcn_readfirstlane(ovw[" << w << "]);\n";
  if (two) {
    o << "#pragma clang loop unroll(disable)\n"
      << "  for (uint32_t it = 0; it < 2u; ++it) {\n"
      << "  const uint64_t tile_id = tile_id0 + it;\n"
      << "  const uint64_t base = it ? base_b : base_a;\n";
    if (swz) o << "  const uint64_t px = it ? px_b : px_a;\n";
    o << "  cs.x = 1; cs.y = 0;\n";
    if (init) emit_init();
  }
  for (const DOp& op : ps.ops) {
    switch (op.type) {
      case DOP_M1G:
        for (int j = 0; j < 4; ++j)
          if ((op.mask >> j) & 1) g.gate(j, op.slot[j]);
        break;
      case DOP_M1: {
        const int j = g.reg_pos(op.a);
        if (j < 0) g.fail("2x2 matrix on a non-register bit");
        else g.gate(j, op.slot[0]);
        break;
      }
      case DOP_DSIGN: g.dsign(op); break;
      case DOP_SFLIP: g.flush_signs(); break;
      case DOP_D1:
        if (frame[op.slot[0]] != FRAME_ABSORB) g.diag(op);  // else merged into a pending phase frame
        break;
      case DOP_D2: g.diag(op); break;
      case DOP_M2: g.m2(op); break;
      case DOP_MR: g.mr(op); break;
      case DOP_KR: g.kr(op); break;
      case DOP_PHASE: g.phase(op); break;
      case DOP_DOT: g.dot(op); break;
      default: g.fail("unknown operation type " + std::to_string(op.type));
    }
    if (!g.ok) return "";
  }
  g.flush_signs();
  for (int j = 0; j < 4; ++j)
    if (g.R[j] != k - 4 + j) g.fail("pass does not end in the load layout");
  if (!g.ok) return "";
  if (g.pending) {
    if (g.cs_neg) o << "  cs.x = -cs.x; cs.y = -cs.y;\n";
    for (const std::string& st : g.sets())
      for (int r = 0; r < 16; ++r) o << "  " << st << r << " = cm(cs, " << st << r << ");\n";
  }
  o << "  V* dstp = a.states + (uint64_t)dst * a.N;\n";
  for (int r = 0; r < 16; ++r) {
    const std::string at = "(" + pos_base + ")" + join + std::to_string(og[r]) + "ull";
    if (nt)
      o << "  stnt(dstp + (" << at << "), " << g.S(r) << ");\n";
    else
      o << "  dstp[" << at << "] = " << g.S(r) << ";\n";
  }
  if (two) {
    if (!init) {
      o << "  if (it == 0u) {\n";
      for (int r = 0; r < 16; ++r) o << "    " << g.S(r) << " = b" << r << ";\n";
      o << "  }\n";
    }
    // the next tile's first LDS write must wait for this tile's last reads
    if (g.tile_read) o << "  __syncthreads();\n";
    o << "  }\n";
  }
  if (dual) {
    o << "  V* ldst = lam + (uint64_t)dst * a.N;\n";
    for (int r = 0; r < 16; ++r) o << "  ldst[(" << pos_base << ")" << join << og[r] << "ull] = l" << r << ";\n";
  }
  o << "}\n";
  *needs_full = g.needs_full;
  return o.str();
}

}  // namespace

std::string jit_pass_source(const Pass& ps, int n, int precision, const std::string& name, bool split,
                            uint32_t* tile_elems, bool dual, int waves, bool swz, bool nt, int tpb,
                            uint32_t* tiles_per_block) {
  bool full = false;
  split = split && !dual;
  if (tpb != 2 || dual || n <= ps.k) tpb = 1;
  std::string src = gen_pass(ps, n, precision, name, split, dual, waves, swz, nt, tpb, &full);
  if (split && full) {  // a 4x4 matrix off the register bits needs the whole tile
    split = false;
    src = gen_pass(ps, n, precision, name, false, dual, waves, swz, nt, tpb, &full);
  }
  if (tile_elems) *tile_elems = src.empty() ? 0u : (1u << (ps.k - (split ? 1 : 0)));
  if (tiles_per_block) *tiles_per_block = (uint32_t)tpb;
  return src;
}

namespace {

ptsbe_status compile_one(const std::string& src, const std::string& name, std::vector<char>& code, std::string& err) {
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), (name + ".hip").c_str(), 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
    err = "hiprtcCreateProgram failed";
    return PTSBE_E_DEVICE;
  }
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops"};
  hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
  if (r != HIPRTC_SUCCESS) {
    size_t ls = 0;
    hiprtcGetProgramLogSize(prog, &ls);
    std::string log(ls, '\0');
    if (ls) hiprtcGetProgramLog(prog, &log[0]);
    err = std::string("pass compiler: ") + hiprtcGetErrorString(r) + ": " + log.substr(0, 2000);
    hiprtcDestroyProgram(&prog);
    return PTSBE_E_DEVICE;
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prog, &cs);
  code.resize(cs);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  return PTSBE_OK;
}

}  // namespace

ptsbe_status jit_build(const Plan& P) {
  JitProgram& J = *P.jit;
  std::lock_guard<std::mutex> lk(J.mu);
  if (J.built) return J.build_status == PTSBE_OK ? PTSBE_OK : fail(J.build_status, J.build_error);
  const auto t0 = std::chrono::steady_clock::now();
  std::map<std::string, int> by_body;
  auto add_program = [&](const std::vector<Pass>& passes, bool dual, std::vector<int>& kernel_of,
                         const char* stem) {
    kernel_of.assign(passes.size(), -1);
    for (size_t p = 0; p < passes.size(); ++p) {
      uint32_t te = 0, tpb = 1;
      const std::string body =
          jit_pass_source(passes[p], P.n, P.precision, "KERNEL_NAME", P.half_tile_lds, &te, dual, P.waves,
                          P.swizzle, P.nontemporal, P.tiles_per_block, &tpb);
      if (body.empty()) continue;
      auto it = by_body.find(body);
      if (it != by_body.end()) {
        kernel_of[p] = it->second;
        continue;
      }
      const int id = (int)J.names.size();
      const std::string name = stem + std::to_string(id);
      std::string src = body;
      src.replace(src.find("KERNEL_NAME"), 11, name);
      by_body[body] = id;
      kernel_of[p] = id;
      J.names.push_back(name);
      J.sources.push_back(src);
      J.tile_elems.push_back(te);
      J.tiles_per_block.push_back(tpb);
    }
  };
  add_program(P.passes, false, J.pass_kernel, "ptsbe_pass_");
  if (P.has_adjoint) add_program(P.adj.passes, true, J.adj_pass_kernel, "ptsbe_adjoint_pass_");
  const size_t K = J.names.size();
  if (const char* dir = std::getenv("PTSBE_PASS_SOURCE_DIR")) {  // inspection: keep the generated sources
    for (size_t i = 0; i < K; ++i) {
      FILE* f = std::fopen((std::string(dir) + "/" + J.names[i] + ".hip").c_str(), "w");
      if (f) {
        std::fwrite(J.sources[i].data(), 1, J.sources[i].size(), f);
        std::fclose(f);
      }
    }
  }
  J.code.assign(K, {});
  std::vector<ptsbe_status> st(K, PTSBE_OK);
  std::vector<std::string> err(K);
  std::atomic<size_t> next{0};
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  // code objects are shared between plans with identical pass sources (process-wide cache)
  static std::mutex cache_mu;
  static std::map<std::string, std::vector<char>> cache;
  auto work = [&]() {
    for (size_t i = next++; i < K; i = next++) {
      {
        std::lock_guard<std::mutex> lk(cache_mu);
        auto it = cache.find(J.sources[i]);
        if (it != cache.end()) {
          J.code[i] = it->second;
          continue;
        }
      }
      st[i] = compile_one(J.sources[i], J.names[i], J.code[i], err[i]);
      if (st[i] == PTSBE_OK) {
        std::lock_guard<std::mutex> lk(cache_mu);
        cache.emplace(J.sources[i], J.code[i]);
      }
    }
  };
  for (unsigned w = 0; w < std::min<size_t>(hw, K); ++w) pool.emplace_back(work);
  for (auto& th : pool) th.join();
  J.compile_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  J.built = true;
  for (size_t i = 0; i < K; ++i)
    if (st[i] != PTSBE_OK) {
      J.build_status = st[i];
      J.build_error = err[i];
      return fail(st[i], err[i]);
    }
  return PTSBE_OK;
}

bool jit_has(const Plan& P, uint32_t pass) {
  return P.jit && P.jit->built && P.jit->build_status == PTSBE_OK && pass < P.jit->pass_kernel.size() &&
         P.jit->pass_kernel[pass] >= 0;
}

namespace {

// Kernel handles of the plan's compiled passes on the current device, loading
// the code objects there at first use.
hipError_t jit_functions(const Plan& P, const std::vector<hipFunction_t>** out) {
  JitProgram& J = *P.jit;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(J.mu);
  auto it = J.functions.find(dev);
  if (it == J.functions.end()) {
    std::vector<hipModule_t> mods(J.code.size());
    std::vector<hipFunction_t> fns(J.code.size());
    for (size_t i = 0; i < J.code.size(); ++i) {
      e = hipModuleLoadData(&mods[i], J.code[i].data());
      if (e != hipSuccess) return e;
      e = hipModuleGetFunction(&fns[i], mods[i], J.names[i].c_str());
      if (e != hipSuccess) return e;
    }
    J.modules[dev] = mods;
    it = J.functions.emplace(dev, fns).first;
  }
  *out = &it->second;
  return hipSuccess;
}

}  // namespace

hipError_t jit_load(const Plan& P) {
  if (!P.jit || !P.jit->built || P.jit->build_status != PTSBE_OK) return hipSuccess;
  const std::vector<hipFunction_t>* fns = nullptr;
  return jit_functions(P, &fns);
}

bool jit_loaded(const Plan& P) {
  if (!P.jit || !P.jit->built || P.jit->build_status != PTSBE_OK) return false;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> lk(P.jit->mu);
  return P.jit->functions.count(dev) != 0;
}

// Dynamic LDS a workgroup may hold on the current device (160 KiB on gfx950).
size_t max_lds_per_block() {
  static std::mutex mu;
  static std::map<int, size_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int v = 0;
  const size_t m = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0
                       ? (size_t)v
                       : 65536;
  cache[dev] = m;
  return m;
}

template <typename V>
hipError_t jit_launch(const Plan& P, uint32_t pass, const PassArgs<V>& a, uint32_t rows, hipStream_t s) {
  const std::vector<hipFunction_t>* fns = nullptr;
  hipError_t e = jit_functions(P, &fns);
  if (e != hipSuccess) return e;
  hipFunction_t f = (*fns)[P.jit->pass_kernel[pass]];
  const Pass& ps = P.passes[pass];
  const uint32_t k = (uint32_t)ps.k, n_slots = (uint32_t)ps.slots.size();
  const size_t te = P.jit->tile_elems[P.jit->pass_kernel[pass]];
  const uint32_t tpb = P.jit->tiles_per_block[P.jit->pass_kernel[pass]];
  const size_t lds = sizeof(V) * (te + lds_mat_entries(ps)) + 4 * ((size_t)n_slots + (n_slots + 31) / 32);
  if (lds > max_lds_per_block()) return hipErrorInvalidConfiguration;
  if (tpb != 1 && (tpb != 2 || P.n <= (int)k)) return hipErrorInvalidConfiguration;
  PassArgs<V> la = a;
  uint32_t slot_begin = 0;
  for (uint32_t p = 0; p < pass; ++p) slot_begin += (uint32_t)P.passes[p].slots.size();
  la.slot_default = a.slot_default + slot_begin;
  void* args[] = {&la};
  return hipModuleLaunchKernel(f, (1u << (P.n - k)) / tpb, rows, 1, 1u << (k - kRegBits), 1, 1, (unsigned)lds, s,
                               args, nullptr);
}

bool jit_has_adjoint(const Plan& P, uint32_t pass) {
  return P.jit && P.jit->built && P.jit->build_status == PTSBE_OK && pass < P.jit->adj_pass_kernel.size() &&
         P.jit->adj_pass_kernel[pass] >= 0;
}

template <typename V>
hipError_t jit_adjoint_launch(const Plan& P, uint32_t pass, const AdjArgs<V>& a, uint32_t rows, hipStream_t s) {
  const std::vector<hipFunction_t>* fns = nullptr;
  hipError_t e = jit_functions(P, &fns);
  if (e != hipSuccess) return e;
  const int kid = P.jit->adj_pass_kernel[pass];
  hipFunction_t f = (*fns)[kid];
  const Pass& ps = P.adj.passes[pass];
  const uint32_t k = (uint32_t)ps.k, n_slots = (uint32_t)ps.slots.size();
  const size_t te = P.jit->tile_elems[kid];
  const size_t lds = sizeof(V) * (te + lds_mat_entries(ps)) + 4 * ((size_t)n_slots + (n_slots + 31) / 32);
  if (lds > 65536) return hipErrorInvalidConfiguration;
  PassArgs<V> la = a.p;
  uint32_t slot_begin = 0;
  for (uint32_t p = 0; p < pass; ++p) slot_begin += (uint32_t)P.adj.passes[p].slots.size();
  la.slot_default = a.p.slot_default + slot_begin;
  V* lam = a.lam;
  double* partial = a.partial;
  uint32_t n_dot = a.n_dot;
  void* args[] = {&la, &lam, &partial, &n_dot};
  return hipModuleLaunchKernel(f, 1u << (P.n - k), rows, 1, 1u << (k - kRegBits), 1, 1, (unsigned)lds, s, args,
                               nullptr);
}

uint32_t jit_adjoint_waves(uint32_t k) {
  const uint32_t bd = 1u << (k - kRegBits);
  return bd > 64 ? bd / 64 : 1u;
}

template hipError_t jit_adjoint_launch<float2>(const Plan&, uint32_t, const AdjArgs<float2>&, uint32_t, hipStream_t);
template hipError_t jit_adjoint_launch<double2>(const Plan&, uint32_t, const AdjArgs<double2>&, uint32_t,
                                                hipStream_t);
template hipError_t jit_launch<float2>(const Plan&, uint32_t, const PassArgs<float2>&, uint32_t, hipStream_t);
template hipError_t jit_launch<double2>(const Plan&, uint32_t, const PassArgs<double2>&, uint32_t, hipStream_t);

}  // namespace ptsbe
