// Host-side objects of the PTSBE library: the execution plan (expanded noisy
// circuit + fused tile passes) and trajectory sets (PTS output).
#pragma once

#include <complex>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/ptsbe.h"
#include "tables.hpp"

namespace ptsbe {

struct JitProgram;

using cd = std::complex<double>;
using Mat = std::vector<cd>;  // row-major d x d

// Thread-local error reporting.
ptsbe_status fail(ptsbe_status st, const std::string& msg);

struct Channel {
  int nq = 1;
  int K = 0;
  std::vector<double> p;       // p_k = tr(K_k^dagger K_k) / d
  std::vector<Mat> U;          // U_k = K_k / sqrt(p_k)
  std::vector<bool> diag;      // U_k diagonal
  bool all_diag = false;
  // 2-qubit channels whose every U_k is a product A_k (x) B_k (B on matrix bit 0):
  bool product = false;
  std::vector<Mat> f0, f1;     // factors on matrix bit 0 / bit 1 (2x2 each)
  // State-dependent 1-qubit channel (not a unitary mixture) whose K_k^dagger K_k
  // are diagonal: p_k = d0[k] P(q = 0) + d1[k] P(q = 1), resolved when the
  // trajectory's state reaches it; U holds the raw Kraus operators.
  bool general = false;
  std::vector<double> d0, d1;
  // A state-dependent channel that is not that case (a 1-qubit channel with
  // non-diagonal K_k^dagger K_k, or any 2-qubit one): p_k = Tr(M_k rho) from the
  // reduced density matrix rho of its qubits, M_k = K_k^dagger K_k.
  bool dense = false;
  std::vector<Mat> M;
};

enum StepKind { ST_GATE, ST_PARAM, ST_SITE, ST_MR, ST_P0, ST_DOT, ST_GCH };

struct Step {
  StepKind kind;
  int nq = 1;
  int q[4] = {0, 0, 0, 0};
  Mat mat;                     // GATE
  bool diag = false;           // diagonal in the computational basis (for every variant)
  bool dagger = false;         // apply the adjoint of the operation (reverse sweep)
  int param = -1, gen = 0;     // PARAM, DOT
  int site = -1;               // SITE
  int mr = -1;                 // MR, GCH: record index
  int chan = -1;               // GCH: channel
  int gidx = -1;               // GCH: index among the state-dependent channel steps
  bool dense = false;          // GCH of a dense channel: decided and applied by its own step
  int dot = -1;                // DOT: index of the gradient contribution
};

struct Site {
  int channel;
  int nq;
  int q[2];
  int step;
  uint32_t op = 0xffffffffu;  // circuit op the site belongs to (none for readout sites)
  uint32_t tag = 0;           // that op's tag
  uint32_t origin = 0;        // PTSBE_SITE_*
};

// One factor of a fused slot: a step, or one half of a product 2-qubit site.
struct Part {
  int step;
  int half;                    // -1: whole step; 0 / 1: factor on the site's first / second qubit
  int emb = -1;                // in a 4x4 slot: 0 / 1 = a 2x2 on the slot's first / second qubit,
                               // 2 = a 4x4 whose qubits are the slot's in swapped order
};

// Phase frames of the forward program.  A diagonal of unit-modulus phases
// commutes with every diagonal operation, so the tables may leave one pending
// on a qubit and let the next matrix on that qubit take it in: a 2x2 slot M
// then runs as V = D^-1 M F, with F the diagonal pending before it and D the
// phases of the diagonal of M F, chosen so that V has a real diagonal (cheaper
// to apply); D stays pending.  A diagonal gate slot between two matrices is
// taken into the pending diagonal and not applied at all.  The chain of every
// qubit ends without a pending diagonal (the last matrix before a measurement,
// a measure-reset or the end of the program absorbs it as a plain 2x2), so
// the states between passes and at the end are the exact ones.
enum FrameRole : uint8_t {
  FRAME_NONE = 0,           // matrix applied as is (a 2x2 or 4x4 slot still absorbs the pending diagonal)
  FRAME_REAL_DIAG = 1,      // 2x2 slot stored as V with a real diagonal; D stays pending
  FRAME_ABSORB = 2,         // unitary diagonal slot with no noise site, merged into the pending
                            // diagonal; the tables hold the identity and the kernels skip it
  FRAME_OVERRIDE_ONLY = 3,  // unitary diagonal 2x2 slot with noise sites: its default becomes the
                            // identity (skipped), a trajectory's override still runs as a 2x2
  FRAME_UNIT_DIAG = 4,      // fixed 2x2 slot stored with a unit diagonal: its whole diagonal,
                            // magnitude included, stays pending (x_r + c x_o per amplitude)
  FRAME_UNIT4 = 5,          // fixed 4x4 slot stored with rows 0..2 of unit diagonal: a product
                            // diagonal d_a (x) d_b stays pending on its two qubits
};

struct Slot {
  uint8_t type;                // DOP_M1 / DOP_M2 / DOP_D1 / DOP_D2
  uint8_t frame = FRAME_NONE;  // FrameRole (forward program only)
  int q[2];                    // global qubits (matrix bit 0, bit 1)
  std::vector<Part> parts;     // applied in order
  std::vector<int> sites;      // sites whose choice changes this slot
  bool uses_params = false;
  bool m2_next[2] = {false, false};  // 4x4: the next non-diagonal operation on matrix bit j's qubit is a matrix
  uint8_t form = 0;            // reverse sweep, 2x2 slots no record changes: 3 real, 4 diagonal for every
                               // parameter value (the compiled sweep applies that form); noise-only slots
                               // whose default is the identity: 5 (applied only where a record overrides
                               // them); 4x4 slots without parameters whose default is a diagonal of +-1: 6
                               // (negations from sign_mask, the matrix only where a record overrides them);
                               // else 0
  uint8_t sign_mask = 0;       // form 6: bit q set where the default's diagonal entry q is -1
};

struct Pass {
  int k = 0;
  std::vector<int> tq;         // tile qubits ascending
  std::vector<int> oq;         // other qubits ascending
  std::vector<DOp> ops;
  std::vector<Slot> slots;
  uint32_t flags = 0;
};

// Execution step: a tile pass, or a decision of a group of record entries
// (measure-resets, or one state-dependent channel), or in the reverse sweep the
// restore of the state checkpointed at a state-dependent channel.
struct ExecStep {
  int pass = -1;               // >= 0: tile pass index
  std::vector<int> mr_qubits;  // decision / restore: qubits
  std::vector<int> mr_index;   // decision / restore: record indices
  bool wall = false;           // a state-dependent channel: every qubit's phase frame ends here
  int restore = -1;            // reverse sweep: checkpoint (state-dependent channel index) to restore
  bool dense = false;          // a dense channel's step: reduced density matrix, decision, application
};

// Decision data of the record entries (measure-resets and state-dependent
// channels), uploaded with every run: rec_chan[r] = offset into chan_param of
// entry r's channel, or 0xffffffff for a measure-reset; rec_gidx[r] = its
// uniform's word; chan_param per channel: K, then d0[0..K), d1[0..K), then the
// K raw Kraus operators (2x2 row-major, re/im interleaved: 8 doubles each).
struct RecordInfo {
  std::vector<uint32_t> rec_chan, rec_gidx;
  std::vector<double> chan_param;
};

// A fused device program: steps, the tile passes and execution steps built
// from them, and the slots each noise site touches.
struct Program {
  std::vector<Step> steps;
  std::vector<Pass> passes;
  std::vector<ExecStep> exec;
  std::vector<std::vector<std::pair<int, int>>> site_slots;
  std::vector<int> dot_param;  // DOT index -> parameter index
  std::vector<int> dot_gen;    // DOT index -> generator
};

struct Plan {
  int n = 0;
  int precision = PTSBE_C64;
  int tile_bits = 12;
  int min_fill = 2;            // phase scheduler: fewest 2x2 matrices worth a partial wave
  int n_params = 0;
  int n_measure = 0;           // record entries: measure-resets and state-dependent channel steps
  int n_general = 0;           // state-dependent channel steps
  RecordInfo rec_info;
  std::vector<Channel> channels;
  std::vector<Step> steps;
  std::vector<Site> sites;
  std::vector<uint32_t> site_off; // offsets into site_p
  std::vector<double> site_p;     // p_{s,k}
  std::vector<Pass> passes;
  std::vector<ExecStep> exec;
  // site -> (pass, slot) list
  std::vector<std::vector<std::pair<int, int>>> site_slots;
  // reverse-sweep program of the adjoint gradient (unitary circuits with parameters)
  bool has_adjoint = false;
  Program adj;
  // per-pass compiled kernels (built on first use unless disabled)
  bool use_jit = true;
  bool half_tile_lds = false;  // compiled passes change registers through half a tile of LDS
  int waves = 0;               // waves per SIMD the compiled passes' register budget is set for (0 = default)
  bool pair_fusion = true;     // diagonal 2-qubit gates merge with the 2x2 runs around them into 4x4 slots
  bool swizzle = true;         // states stored at swizzle(x) (kernels.hpp)
  bool nontemporal = false;    // compiled passes load and store the states with nontemporal hints
  int tiles_per_block = 1;     // tiles of a state one workgroup of a compiled forward pass runs
  bool tile_search = true;     // each pass's tile: the best of the greedy one and qubit windows
  std::shared_ptr<JitProgram> jit;
};

struct TrajSet {
  std::shared_ptr<const Plan> plan;
  uint64_t alpha0 = 0;
  std::vector<uint64_t> m;
  std::vector<double> p;
  std::vector<uint64_t> count;
  std::vector<uint32_t> rec_off;   // n_traj + 1
  std::vector<uint32_t> rec_site;
  std::vector<uint8_t> rec_kraus;
  uint64_t total_shots = 0;
  uint64_t total_count = 0;
  // Unnormalised ensemble weight of each trajectory, the proportions its shots
  // are allocated by: the draw count (multiplicity allocation), p_alpha
  // (reweight), 1 (uniform and per-shot), m_alpha (caller records).  The
  // expectation E = sum_alpha w_alpha <O>_alpha and its gradient use
  // w_alpha = wbasis_alpha / sum over the set.
  std::vector<double> wbasis;
  // Cached device tables (host copy), keyed by the parameter values they used.
  std::mutex mu;
  std::vector<double> cached_params;
  std::vector<uint8_t> table_blob;
  TableLayout layout{};
  bool table_valid = false;
  size_t pool_elems = 0;
  std::vector<uint64_t> chunk_off;
  uint32_t cached_chunk = 0;
  // the same for the adjoint (reverse-sweep) program
  std::vector<double> adj_params;
  std::vector<uint8_t> adj_blob;
  TableLayout adj_layout{};
  bool adj_valid = false;
  std::vector<uint8_t> adj_aux;    // host staging of weights and the dot -> parameter map
  std::vector<uint32_t> route_host; // host staging of prefix-sharing launch routes (src, dst pairs)
  std::vector<double> weights_host; // host staging of the ensemble weights (expectation mode)
  std::vector<uint32_t> route_off;
  std::vector<uint32_t> eff_host;   // host staging of each trajectory's first own execution step (prefix sharing)
  std::vector<uint64_t> uq_host;    // host staging of the distinct-shot pass's offset arrays
};

// Normalised ensemble weights w_alpha = wbasis_alpha / sum (summed in trajectory order).
std::vector<double> ensemble_weights(const TrajSet& ts);

// Prefix sharing of the forward program (run.cpp): whether it applies to a run
// of `ts` with options `o` (flags only), and the launch routes of the batch
// [b0, b0 + bb): (source slot, destination slot) pairs per execution step,
// step e's at out[2 off[e] .. 2 off[e + 1]), each trajectory's first own step
// appended to eff_out.
bool prefix_sharing(const Plan& P, const TrajSet& ts, const ptsbe_run_opts* o);
void build_routes(const Plan& P, const TrajSet& ts, uint32_t b0, uint32_t bb, std::vector<uint32_t>& out,
                  std::vector<uint32_t>& off, std::vector<uint32_t>& eff_out);

// Matrix helpers
Mat mat_identity(int d);
Mat mat_mul(const Mat& a, const Mat& b, int d);        // a * b
bool mat_is_diag(const Mat& a, int d, double tol = 0.0);
Mat rot_matrix(int gen, double theta);

// Slot matrix for a trajectory: choice(site) gives its Kraus index.  `steps` is
// the step list of the program the slot belongs to.
Mat slot_matrix(const Plan& plan, const std::vector<Step>& steps, const Slot& s, const double* params,
                const std::map<int, int>& choice);

// Phase frames: per slot of a program, the pending diagonal it takes in
// (`in[j]` for its matrix qubit j) and, for FRAME_REAL_DIAG, the diagonal it
// leaves pending (`out`).  Computed from the slots' default matrices.
struct SlotFrame {
  cd in[2][2] = {{cd(1, 0), cd(1, 0)}, {cd(1, 0), cd(1, 0)}};
  cd out[2] = {cd(1, 0), cd(1, 0)};   // 2x2, or a 4x4's matrix bit 0 (FRAME_UNIT4)
  cd out2[2] = {cd(1, 0), cd(1, 0)};  // a 4x4's matrix bit 1 (FRAME_UNIT4)
};
std::vector<std::vector<SlotFrame>> slot_frames(int n, const std::vector<Pass>& passes,
                                                const std::vector<ExecStep>& exec,
                                                const std::vector<std::vector<Mat>>& defaults);
// The matrix a slot's table entry holds for true matrix M (default or override).
Mat frame_matrix(const Slot& s, const SlotFrame& f, const Mat& M);

// Pauli twirl of a channel: probabilities of the 4^nq Pauli strings (digit j of
// the string index, 0 I / 1 X / 2 Y / 3 Z, on matrix bit j).
std::vector<double> pauli_twirl_probs(const std::vector<Mat>& K, int nq);
ptsbe_status pauli_twirl_channel(uint32_t nq, const double* kraus, uint32_t n_kraus, double* probs);

// Planner
ptsbe_status build_plan(const ptsbe_circuit* c, const ptsbe_noise_model* nm,
                        const ptsbe_plan_opts* o, std::shared_ptr<Plan>* out);

// Build the device tables of a trajectory set (cached in ts).
ptsbe_status build_tables(TrajSet& ts, const double* params, uint32_t chunk);
// Device tables of the adjoint (reverse-sweep) program, cached in ts.
ptsbe_status build_adj_tables(TrajSet& ts, const double* params);

// Distinct shots per trajectory and (basis index, count) pairs (unique.hip).
ptsbe_status unique_workspace_size(const TrajSet& ts, uint32_t max_batch, size_t* bytes);
ptsbe_status unique_shots(TrajSet& ts, const void* d_bits, void* d_ws, size_t ws_bytes, uint64_t* d_unique,
                          void* d_pair_index, uint32_t* d_pair_count, hipStream_t s);

}  // namespace ptsbe

struct ptsbe_plan_s {
  std::shared_ptr<ptsbe::Plan> plan;
};
struct ptsbe_trajset_s {
  std::shared_ptr<ptsbe::TrajSet> ts;
};
struct ptsbe_graph_s {
  std::shared_ptr<const ptsbe::Plan> plan;
  std::shared_ptr<ptsbe::TrajSet> ts;
  hipGraphExec_t exec = nullptr;
};
