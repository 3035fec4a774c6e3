/*
 * ptsbe.h -- C ABI of the PTSBE hot path on MI355X (gfx950).
 *
 * Pre-Trajectory Sampling with Batched Execution (arXiv 2504.16297):
 *   1. PTS (Sec. 3.1): choose whole Kraus-operator sequences alpha and a shot
 *      count m_alpha for each, before any state is simulated.
 *   2. BE (Sec. 3): prepare each fixed-Kraus state once on the GPU, then draw
 *      all m_alpha bitstrings from |psi_alpha|^2 in bulk; each shot carries
 *      the id of its trajectory, whose error record is kept on the host
 *      (Sec. 1, third innovation: error provenance as lightweight metadata).
 *
 * Conventions
 *  - Basis index x = sum_q x_q 2^q (qubit 0 is the least significant bit).
 *    A k-qubit matrix acting on qubits (q_0..q_{k-1}) has row/column bit j
 *    <-> qubit q_j.  Matrices are complex128, row-major, interleaved (re, im).
 *  - Every call returns a ptsbe_status; on error nothing has been enqueued on
 *    the stream, outputs are undefined and ptsbe_last_error() (thread-local)
 *    explains.  No C++ exception crosses this boundary.
 *  - Handles (plans, trajectory sets) are library-owned host objects,
 *    immutable after creation, shareable across threads, freed by their
 *    destroy call.  A handle must outlive the stream work enqueued with it.
 *  - Every device buffer (workspace, outputs, uniforms) is owned by the
 *    caller.  The library never allocates device memory (the one fixed device
 *    array of ptsbe_run_batch_noalloc is part of its code object).
 *  - Device launches are asynchronous on the caller's hipStream_t (passed as
 *    void*; NULL is the null stream).  Device-side conditions (a
 *    non-deterministic measure-reset) are written to a status word in the
 *    workspace; ptsbe_run_status() waits for the stream and reads it.
 */
#ifndef PTSBE_H
#define PTSBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PTSBE_OK = 0,
    PTSBE_E_ARG = 1,            /* invalid argument: null pointer, bad qubit, size mismatch */
    PTSBE_E_NOT_CPTP = 2,       /* a channel violates sum_k K_k^dagger K_k = I (Sec. 2.2) beyond 1e-12 */
    PTSBE_E_UNSUPPORTED = 3,    /* valid but not implemented (a channel neither a unitary mixture nor
                                   resolvable from one qubit's populations, n > 35) */
    PTSBE_E_CAPACITY = 4,       /* output capacity below the total shot count */
    PTSBE_E_OOM = 5,            /* workspace smaller than ptsbe_workspace_size() */
    PTSBE_E_DEVICE = 6,         /* a HIP call failed */
    PTSBE_E_NONDET_MEASURE = 7  /* a measure-reset outcome was not deterministic (device status) */
} ptsbe_status;

/* Thread-local description of the last error of this thread. */
const char* ptsbe_last_error(void);
/* Library version string. */
const char* ptsbe_version(void);

/* ------------------------------------------------------------------ circuit */

enum {
    PTSBE_OP_GATE = 0,          /* fixed matrix `mat` on q[0..nq-1], nq <= 4 */
    PTSBE_OP_PARAM = 1,         /* exp(-i theta P / 2) on q[0], theta = params[index], P = gen */
    PTSBE_OP_NOISE = 2,         /* explicit noise site: channel `index` on q[0..nq-1] */
    PTSBE_OP_MEASURE_RESET = 3, /* mid-circuit measure of q[0] (recorded), then reset to |0> */
    PTSBE_OP_PROJECT0 = 4       /* apply |0><0| on q[0] and renormalise (no record) */
};
enum { PTSBE_GEN_X = 1, PTSBE_GEN_Y = 2, PTSBE_GEN_Z = 3 };

typedef struct {
    uint32_t kind;              /* PTSBE_OP_* */
    uint32_t nq;                /* number of qubits the op acts on (1..4; 1 for PARAM/MR/PROJECT0) */
    uint32_t q[4];              /* distinct qubits, each < n_qubits */
    const double* mat;          /* GATE: 2^nq x 2^nq complex128, read during ptsbe_plan only */
    int32_t index;              /* PARAM: parameter index; NOISE: channel index */
    uint32_t gen;               /* PARAM: PTSBE_GEN_X/Y/Z */
    uint32_t tag;               /* caller's gate-type tag, matched by PTSBE_ATTACH_AFTER_TAG rules */
    uint32_t reserved;
} ptsbe_op;

typedef struct {
    uint32_t n_qubits;          /* 1..35 (35: a 256 GiB complex64 state) */
    uint32_t n_ops;
    const ptsbe_op* ops;
} ptsbe_circuit;

/* ------------------------------------------------------------- noise model */

/* A channel {K_0 .. K_{n_kraus-1}} on nq (1 or 2) qubits: n_kraus consecutive
 * 2^nq x 2^nq complex128 matrices.  It must be CPTP (Sec. 2.2).  A unitary
 * mixture, K_k^dagger K_k = p_k I (Sec. 2.2 feature 2, read as
 * K_k = sqrt(p_k) U_k), has state-independent p_k: its sites are pre-sampled
 * by PTS, and K_0 is taken as the "no error" operator of the record.  Any
 * other channel is resolved from the state when a trajectory reaches it
 * (Algorithm 1's state-dependent branch; see ptsbe_plan_get_record_info), or
 * replaced by its Pauli twirl with PTSBE_PLAN_TWIRL.
 * At most 16 operators per channel. */
typedef struct {
    uint32_t nq;
    uint32_t n_kraus;
    const double* kraus;
} ptsbe_channel;

enum {
    PTSBE_ATTACH_AFTER_TAG = 0,      /* a site after every GATE/PARAM op with op.tag == tag, on its qubits */
    PTSBE_ATTACH_BEFORE_MEASURE = 1, /* a site before every MEASURE_RESET, on its qubit */
    PTSBE_ATTACH_BEFORE_READOUT = 2  /* at the end, one site per qubit set in qmask, ascending */
};

typedef struct {
    uint32_t when;
    uint32_t tag;
    uint32_t channel;
    uint32_t reserved;
    uint64_t qmask;
} ptsbe_attach;

typedef struct {
    uint32_t n_channels;
    const ptsbe_channel* channels;
    uint32_t n_rules;
    const ptsbe_attach* rules;
} ptsbe_noise_model;

/* Site order ("NoisyCircuit" of Algorithm 2): walking the ops in order, the
 * BEFORE_MEASURE sites of an MEASURE_RESET come before it (rule order); an
 * explicit NOISE op is a site at its position; AFTER_TAG sites follow their
 * op (rule order); BEFORE_READOUT sites come last (rule order, then qubit). */

/* -------------------------------------------------------------------- plan */

enum { PTSBE_C64 = 0, PTSBE_C128 = 1 };

typedef struct {
    uint32_t precision;         /* PTSBE_C64 (FP32 state) or PTSBE_C128 (FP64 state) */
    uint32_t tile_qubits;       /* 0 = automatic; else qubits per LDS tile (4..13) */
    uint32_t flags;             /* bits 0..2: fewest 2x2 matrices per register group worth a
                                   partial group (0 = 2); PTSBE_PLAN_NO_COMPILE,
                                   PTSBE_PLAN_HALF_TILE_LDS, PTSBE_PLAN_NO_PHASE_FRAMES;
                                   bits 8..11: waves per SIMD (PTSBE_PLAN_WAVES_SHIFT) */
    uint32_t reserved;
} ptsbe_plan_opts;

/* Run every pass through the generic (interpreting) tile kernels instead of
 * the per-pass kernels the plan compiles for itself (see ptsbe_plan_compile). */
#define PTSBE_PLAN_NO_COMPILE 8u
/* Compiled passes move amplitudes between register sets through half a tile
 * of LDS in two rounds (more resident workgroups per CU, two more barriers
 * per register change). */
#define PTSBE_PLAN_HALF_TILE_LDS 16u
/* Keep every slot matrix as it is.  By default the planner rewrites the
 * forward program in phase frames: a unit-modulus diagonal may stay pending
 * on a qubit between two of its matrices (it commutes with every diagonal
 * operation in between), so that a 2x2 matrix is stored with a real diagonal
 * (cheaper in the compiled passes) and diagonal gates between two matrices are
 * merged away.  The states between passes and at the end are unchanged. */
#define PTSBE_PLAN_NO_PHASE_FRAMES 32u
/* flags bits 8..11: the number of waves per SIMD (1..8) the compiled passes'
 * register budget is set for (512 / waves VGPRs, the compiler spills beyond
 * it); 0 leaves the budget of the forward passes to the compiler and sets
 * three waves for the reverse sweep of the adjoint gradient (psi and lambda
 * in registers).  Each pass kernel holds its
 * 4096-amplitude tile (32 KiB in complex64) in LDS, so up to 5 workgroups fit
 * a compute unit. */
#define PTSBE_PLAN_WAVES_SHIFT 8u
/* Replace every channel that is not a unitary mixture (amplitude damping, ...)
 * by its Pauli twirl (see ptsbe_pauli_twirl), which is: Pauli-twirled noise
 * models, one of the tailored error models Sec. 1 names.  Without the flag such
 * channels are resolved from the state (see ptsbe_plan_get_record_info). */
#define PTSBE_PLAN_TWIRL 64u
/* Plan flag: no pair fusion.  By default a diagonal 2-qubit gate (CZ, ...)
 * whose two qubits both carry a pending run of 1-qubit operations merges with
 * them into one 4x4 slot, which also takes the following 1-qubit operations on
 * either qubit until another operation needs one of them (in a brick circuit one
 * 4x4 then replaces four 2x2 matrices and a sign flip). */
#define PTSBE_PLAN_NO_PAIR_FUSION 128u
/* Plan flags: state storage order.  Swizzled storage puts amplitude x of a
 * state of more than 2^12 amplitudes at x XOR (f(x >> 12) << 4), f a fixed
 * linear map of the high index bits to 8 bits: runs of 16 amplitudes and blocks
 * of 4096 stay in place, but the runs a tile pass moves no longer differ only in
 * high address bits (faster on the HBM for large states, slower for small
 * ones).  By default states of PTSBE_SWIZZLE_MIN_QUBITS qubits or more are
 * swizzled; NO_SWIZZLE keeps every state in plain index order, SWIZZLE swizzles
 * every state above 12 qubits.  States leave the library in plain order either
 * way (STATES mode, shots, expectation values). */
#define PTSBE_PLAN_NO_SWIZZLE 4096u
#define PTSBE_PLAN_SWIZZLE 8192u
#define PTSBE_SWIZZLE_MIN_QUBITS 22u
/* Plan flag: the compiled passes load and store the states with nontemporal
 * (streaming) cache hints. */
#define PTSBE_PLAN_NONTEMPORAL 16384u
/* Plan flag: each workgroup of a compiled forward pass runs two tiles of its
 * state, one after the other, with the second tile's loads issued before the
 * first tile's arithmetic (twice the state bytes in flight per workgroup, one
 * matrix set-up for both). */
#define PTSBE_PLAN_TWO_TILES 32768u
/* Plan flag: no tile search.  By default the scheduler builds each pass's tile
 * both by taking operations greedily in circuit order and from every window of
 * consecutive qubits beside the always-present lowest ones (as wide as the
 * tile's free part or two qubits narrower), and keeps the tile that runs the
 * most non-diagonal operations, counting the best take of the pass after it
 * too (on brick circuits a window follows a light cone through many layers:
 * about half the passes). */
#define PTSBE_PLAN_NO_TILE_SEARCH 65536u

typedef struct ptsbe_plan_s* ptsbe_plan_t;
typedef struct ptsbe_trajset_s* ptsbe_trajset_t;

typedef struct {
    uint32_t n_qubits;
    uint32_t n_sites;           /* noise sites after rule expansion */
    uint32_t n_params;          /* 1 + largest PARAM index, 0 if none */
    uint32_t n_measure;         /* MEASURE_RESET ops (record length per trajectory) */
    uint32_t n_passes;          /* fused state passes (tile kernels) per trajectory */
    uint32_t n_steps;           /* passes + measurement steps */
    uint32_t precision;
    uint32_t tile_qubits;
    uint32_t max_kraus;         /* largest channel size */
    uint32_t total_kraus;       /* sum over sites of the channel size */
    uint32_t swizzled;          /* 1: the plan's states are stored swizzled (PTSBE_PLAN_SWIZZLE) */
} ptsbe_plan_info;

/* Validate a circuit and noise model and build the execution plan: expand the
 * noise rules into sites, check CPTP and the unitary-mixture form of every
 * channel, and fuse the operations into tile passes.  `opts` may be NULL.
 * The matrices are copied; the caller's arrays may be freed afterwards. */
ptsbe_status ptsbe_plan(const ptsbe_circuit* circuit, const ptsbe_noise_model* noise,
                        const ptsbe_plan_opts* opts, ptsbe_plan_t* out);
ptsbe_status ptsbe_plan_get_info(ptsbe_plan_t plan, ptsbe_plan_info* out);
/* Compile the plan's tile passes into their own gfx950 kernels (hiprtc; host
 * only, no device needed): each pass's operation list is unrolled into
 * straight-line register code, structurally equal passes share a kernel.
 * ptsbe_run_batch calls this on first use; calling it first moves the cost
 * (about a second per distinct pass, in parallel threads) out of the run.
 * *n_kernels / *seconds (optional) receive the kernel count and compile time.
 * PTSBE_E_DEVICE carries the compiler log if compilation fails. */
ptsbe_status ptsbe_plan_compile(ptsbe_plan_t plan, uint32_t* n_kernels, double* seconds);
/* Inspection: the generated HIP source of pass `pass` (kernel symbol
 * "ptsbe_pass") of the forward program, or with adjoint != 0 of the adjoint
 * gradient's reverse sweep (signature (args, lambda, partial, n_dot)),
 * NUL-terminated; an empty string if that pass runs through the generic
 * kernels.  With out == NULL only *len (bytes including the NUL) is set. */
ptsbe_status ptsbe_plan_pass_source(ptsbe_plan_t plan, uint32_t pass, uint32_t adjoint, char* out,
                                    size_t* len);
/* Per-site probabilities p_{s,k}: offsets[n_sites+1] into probs[total_kraus];
 * qubits[2*n_sites] (second entry 0xffffffff for 1-qubit sites); either may be NULL. */
ptsbe_status ptsbe_plan_get_sites(ptsbe_plan_t plan, uint32_t* offsets, double* probs,
                                  uint32_t* qubits);
/* Where each noise site comes from: op_index[s] = the circuit op it follows
 * (AFTER_TAG), precedes (BEFORE_MEASURE) or is (an explicit NOISE op), or
 * 0xffffffff for BEFORE_READOUT sites; tag[s] = that op's tag (0 otherwise);
 * origin[s] = PTSBE_SITE_*.  Each array has n_sites entries; any may be NULL. */
enum { PTSBE_SITE_NOISE_OP = 0, PTSBE_SITE_AFTER_TAG = 1, PTSBE_SITE_BEFORE_MEASURE = 2,
       PTSBE_SITE_BEFORE_READOUT = 3 };
ptsbe_status ptsbe_plan_get_site_ops(ptsbe_plan_t plan, uint32_t* op_index, uint32_t* tag, uint32_t* origin);
/* The record entries of a trajectory (n_measure of them, in circuit order):
 * measure-resets (outcome bit) and state-dependent channel steps (chosen Kraus
 * index).  channel[r] = the entry's channel index, or 0xffffffff for a
 * measure-reset; gidx[r] = the word of the channel decision's uniform in the
 * stream [seed, 4 << 56 | cfg << 48 | alpha] (0 for measure-resets).  A
 * state-dependent channel is a 1- or 2-qubit channel that is not a unitary
 * mixture: it is resolved when the trajectory's state reaches it (Algorithm
 * 1's state-dependent branch), with p_k = <psi|K_k^dagger K_k|psi> / <psi|psi>
 * and k the smallest index with u < p_0 + ... + p_k (the last with p_k > 0
 * past the end), then K_k / sqrt(p_k).  With diagonal K_k^dagger K_k on one
 * qubit (amplitude damping) p_k comes from the qubit's populations and K_k is
 * applied in the next tile pass; otherwise from the FP64 reduced density
 * matrix of the channel's qubits, in a step of its own that also applies K_k.
 * Arrays have n_measure entries; either may be NULL. */
ptsbe_status ptsbe_plan_get_record_info(ptsbe_plan_t plan, uint32_t* channel, uint32_t* gidx);
void ptsbe_plan_destroy(ptsbe_plan_t plan);

/* ---------------------------------------------------- pre-trajectory sampling */

enum {
    PTSBE_PTS_PROPORTIONAL = 0, /* per site one exact categorical draw: records appear with p_alpha */
    PTSBE_PTS_ALG2_LITERAL = 1, /* Algorithm 2 as printed (r <= p per operator, first compatible wins) */
    PTSBE_PTS_MOST_LIKELY = 2,  /* the k_max records of highest joint probability (Sec. 3.1) */
    PTSBE_PTS_PER_SHOT = 3      /* conventional trajectories (Algorithm 1): one undeduplicated draw per shot */
};
enum {
    PTSBE_ALLOC_MULTIPLICITY = 0, /* m_alpha = count_alpha * total_shots / n_draws, largest remainder */
    PTSBE_ALLOC_REWEIGHT = 1,     /* m_alpha ~ p_alpha / sum_selected p_beta (Sec. 3.1), largest remainder */
    PTSBE_ALLOC_UNIFORM = 2       /* m_alpha = nshots for every record (Algorithm 2) */
};

typedef struct {
    uint32_t mode;              /* PTSBE_PTS_* */
    uint32_t alloc;             /* PTSBE_ALLOC_* (PER_SHOT forces one shot per draw) */
    uint64_t n_draws;           /* PROPORTIONAL, ALG2_LITERAL, PER_SHOT */
    uint64_t k_max;             /* MOST_LIKELY */
    uint64_t total_shots;       /* MULTIPLICITY, REWEIGHT */
    uint64_t nshots;            /* UNIFORM */
    uint64_t seed;              /* first Philox key word */
    uint32_t cfg;               /* workload id, bits 48..55 of the second key word */
    uint32_t stream;            /* 0: default (1 = PTS, 3 = PER_SHOT); bits 56..63 of the key */
    double p_min, p_max;        /* probability band on p_alpha; both 0 = no band (Sec. 3.1) */
    /* Selection criteria (Sec. 3.1: criteria on gate type, parity, location added
     * to the choice of each operator in Algorithm 2).  kraus_allow: NULL, or one
     * flag per (site, Kraus index) in the order of ptsbe_plan_get_sites; an
     * operator k >= 1 whose flag is 0 is never chosen (its site keeps operator
     * 0: in PROPORTIONAL / PER_SHOT a draw of it counts as operator 0, in
     * ALG2_LITERAL its test is skipped, MOST_LIKELY never enumerates it).  Build
     * the flags from ptsbe_plan_get_site_ops (the op and tag a site belongs
     * to, i.e. gate type and location) and the Kraus index (error type). */
    const uint8_t* kraus_allow;
    uint32_t min_errors;        /* records with fewer operators k >= 1 are dropped */
    uint32_t max_errors;        /* records with more are dropped; 0 = no limit */
    uint32_t error_parity;      /* PTSBE_PARITY_*: keep records with any / an even / an odd number */
    uint32_t reserved;
} ptsbe_pts_opts;

enum { PTSBE_PARITY_ANY = 0, PTSBE_PARITY_EVEN = 1, PTSBE_PARITY_ODD = 2 };

/* Selection flags for ptsbe_pts_opts.kraus_allow from site properties (Sec. 3.1:
 * criteria on gate type, location and error type added to the choice of each
 * operator).  Operator k >= 1 of site s is allowed when the tag of the op the
 * site belongs to is in tags (gate type), every qubit of the site is in qubits
 * and its op index in ops (location), its origin (PTSBE_SITE_*) in origins, and
 * k in kraus (error type); a NULL list accepts anything.  Operators k = 0 are
 * always flagged 1.  flags: caller-owned host array of total_kraus bytes
 * (ptsbe_plan_info), in the order of ptsbe_plan_get_sites. */
typedef struct {
    const uint32_t* tags;    uint32_t n_tags;
    const uint32_t* qubits;  uint32_t n_qubits;
    const uint32_t* ops;     uint32_t n_ops;
    const uint32_t* origins; uint32_t n_origins;
    const uint32_t* kraus;   uint32_t n_kraus;
} ptsbe_site_filter;
ptsbe_status ptsbe_site_selection(ptsbe_plan_t plan, const ptsbe_site_filter* filter, uint8_t* flags);

/* Run a PTS algorithm (Sec. 3.1).  Draw t of PROPORTIONAL uses the Philox4x64-10
 * stream keyed [seed, stream<<56 | cfg<<48 | t]; its word s (NumPy's raw order:
 * counter block s/4 + 1, word s%4) gives site s the uniform (word >> 11) 2^-53
 * and k_s = the smallest k with u < p_0 + ... + p_k.  Equal records merge
 * (uniqueKraus) in order of first appearance. */
ptsbe_status ptsbe_sample_kraus(ptsbe_plan_t plan, const ptsbe_pts_opts* opts,
                                ptsbe_trajset_t* out);
/* A trajectory set from caller records: rec_off[n_traj+1] into rec_site/rec_kraus
 * (site ids ascending within a record, kraus index >= 1), m[n_traj] shots each.
 * p_alpha is recomputed; counts are 1.  alpha0 is the global id of record 0. */
ptsbe_status ptsbe_trajset_from_records(ptsbe_plan_t plan, uint32_t n_traj, const uint32_t* rec_off,
                                        const uint32_t* rec_site, const uint8_t* rec_kraus,
                                        const uint64_t* m, uint64_t alpha0, ptsbe_trajset_t* out);
/* Trajectories [begin, end) as a new set that keeps their global ids, so the
 * counter-based sampler reproduces them bit for bit (resume by range). */
ptsbe_status ptsbe_trajset_slice(ptsbe_trajset_t ts, uint32_t begin, uint32_t end,
                                 ptsbe_trajset_t* out);
/* Query a trajectory set.  Scalars may be NULL; arrays are caller-owned host
 * arrays of n_traj (m, p, count), n_traj+1 (rec_off) or n_entries (rec_site,
 * rec_kraus) elements, or NULL to skip. */
ptsbe_status ptsbe_trajset_get(ptsbe_trajset_t ts, uint32_t* n_traj, uint64_t* total_shots,
                               uint32_t* n_entries, uint64_t* alpha0, uint64_t* m, double* p,
                               uint64_t* count, uint32_t* rec_off, uint32_t* rec_site,
                               uint8_t* rec_kraus);
/* Ensemble weights of a trajectory set: w[alpha] = b_alpha / sum_beta b_beta
 * (n_traj FP64 values, caller-owned host array), with b_alpha the proportion its
 * shots are allocated by -- the draw count for MULTIPLICITY (so E estimates
 * the channel's expectation without bias), p_alpha for REWEIGHT (the
 * probability-weighted expectation over the selected records, Sec. 3.1), 1 for
 * UNIFORM and PER_SHOT, m_alpha for ptsbe_trajset_from_records; a slice keeps
 * its trajectories' b.  The expectation mode's ensemble value and
 * ptsbe_adjoint_grad use these weights. */
ptsbe_status ptsbe_trajset_weights(ptsbe_trajset_t ts, double* w);
void ptsbe_trajset_destroy(ptsbe_trajset_t ts);

/* ------------------------------------------------------- batched execution */

enum {
    PTSBE_RUN_SHOTS = 0,        /* prepare, then sample m_alpha shots per trajectory */
    PTSBE_RUN_STATES = 1,       /* prepare, normalise, copy states to d_state_out */
    PTSBE_RUN_EXPECTATION = 2,  /* prepare, then <O>_alpha per trajectory (diagonal O) */
    PTSBE_RUN_ADJOINT = 3       /* workspace query only: ptsbe_adjoint_grad (uses params, max_batch) */
};

typedef struct {
    uint32_t mode;              /* PTSBE_RUN_* */
    uint32_t cfg;               /* sampler key: [seed, 2<<56 | cfg<<48 | alpha] */
    uint64_t seed;
    uint32_t sort_chunk;        /* shots sorted per chunk: power of two, 256..4096 (0 = 4096) */
    uint32_t max_batch;         /* trajectories resident at once (0 = as many as fit) */
    const double* d_uniforms;   /* optional device FP64 uniforms, one per shot in output order */
    const double* params;       /* host array of n_params values (NULL if none) */
    void* d_state_out;          /* STATES: n_traj x 2^n amplitudes (complex64 / complex128) */
    double* d_expval;           /* EXPECTATION: n_traj FP64 values */
    const double* obs_coef;     /* EXPECTATION: n_terms coefficients (host) */
    const uint64_t* obs_zmask;  /* EXPECTATION: n_terms Z-string qubit masks (host) */
    uint32_t n_terms;
    uint32_t flags;             /* PTSBE_RUN_NO_PREFIX_SHARING: every trajectory runs every pass */
    double* timing;             /* optional host array[10]: measured with HIP events on `stream`
                                   (the call then waits for the stream): [0] ms in tile passes,
                                   [1] pass launches, [2] ms in measure-reset steps, [3] ms in
                                   norm/CDF scans, [4] ms in the sampler, [5] ms total,
                                   [6] state bytes moved by the passes (2 x state size per loaded
                                   state-pass, 1 x for the initialising pass), [7] sampler
                                   launches, [8] useful FLOPs of the passes (per amplitude: 14 per
                                   2x2 matrix, 30 per 4x4, 6 per diagonal), [9] state-passes run */
    double* d_ensemble;         /* EXPECTATION: optional device FP64 scalar, receives the ensemble
                                   value E = sum_alpha w_alpha <O>_alpha (w from ptsbe_trajset_weights),
                                   summed on the device in trajectory order */
} ptsbe_run_opts;

/* Prefix sharing (default for plans without state-dependent channels whose
 * first step is a pass from |0> and whose last step is a pass): a trajectory's
 * passes before the first one its noise record changes are not run for it;
 * one error-free state (double-buffered, two extra states of workspace) is
 * carried through those passes and each trajectory's first own pass reads it.
 * A measure-reset decision (outcome [p1 > 1/2], Sec. 2.2's general Kraus
 * branch) is taken once for the carried state and copied to the trajectories
 * still on it.  Results, records included, are bit-identical to running every
 * pass for every trajectory. */
#define PTSBE_RUN_NO_PREFIX_SHARING 1u
/* Sampler support lists (default for states of at most 2^21 amplitudes): the
 * CDF scan also lists, per state, the elements an upper-bound search can return
 * (at most 1024 of them, else the list is not used); a chunk of such a
 * trajectory's shots is then drawn by searching each uniform in that list and
 * writing the per-element counts as ascending runs, which is the sorted
 * chunk's result without the sort.  Shots are bit-identical either way; this
 * flag turns the lists off. */
#define PTSBE_RUN_NO_SUPPORT_LISTS 2u

/* Device workspace in bytes needed by ptsbe_run_batch, or with
 * opts->mode == PTSBE_RUN_ADJOINT by ptsbe_adjoint_grad (max_batch bounds the
 * trajectories whose psi and lambda are resident together; 0 = all). */
ptsbe_status ptsbe_workspace_size(ptsbe_plan_t plan, ptsbe_trajset_t ts, const ptsbe_run_opts* opts,
                                  size_t* bytes);

/* Batched execution (Sec. 3, BE): every trajectory's state is prepared once
 * by the gfx950 tile kernels, normalised, turned into an FP64 cumulative
 * distribution (in place), and its m_alpha shots are drawn by an upper-bound
 * search of sorted uniforms.  Output j of trajectory alpha lands at
 * shot_offset(alpha) + j with shot_offset the exclusive prefix sum of m:
 * d_bits[j] is the basis index (uint32 if n <= 32, else uint64), d_traj[j]
 * the global trajectory id.  d_mr_bits (optional, n_traj x n_measure bytes)
 * receives each trajectory's measure-reset record.  All device pointers are
 * caller-owned; the call only enqueues work on `stream`.  An empty trajectory
 * set enqueues only the clearing of the workspace's status word and returns
 * PTSBE_OK, except in expectation mode with d_ensemble set (PTSBE_E_ARG: the
 * ensemble value has no weights). */
ptsbe_status ptsbe_run_batch(ptsbe_plan_t plan, ptsbe_trajset_t ts, const ptsbe_run_opts* opts,
                             void* d_ws, size_t ws_bytes, void* d_bits, uint32_t* d_traj,
                             uint64_t capacity, uint8_t* d_mr_bits, void* stream);

/* ptsbe_run_batch without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same plan, trajectory set, options and outputs as
 * ptsbe_run_batch, but no workspace argument: the workspace is a fixed device
 * array of PTSBE_NOALLOC_SCRATCH_BYTES inside this library (one per device,
 * held from the first call on that device until the process ends).  The batch
 * is split into the largest groups of trajectories that fit it; a plan whose
 * single trajectory does not fit (about 2^22 amplitudes or more in complex64)
 * fails with PTSBE_E_OOM before anything is enqueued.  The call allocates
 * nothing (no hipMalloc / hipFree, no module load): the plan's compiled pass
 * kernels run only if an earlier ptsbe_run_batch call loaded them on this
 * device, otherwise the generic tile kernels run the same tables (same results).
 * opts->timing must be NULL.  d_status (optional, device, one uint32) receives
 * the run's status word: bit 0 set = a measure-reset outcome was not
 * deterministic (what ptsbe_run_status reports as PTSBE_E_NONDET_MEASURE).
 * Every call on a device shares that device's array and leaves its contents
 * behind: calls that overlap on one device (other streams, other threads)
 * race and must be serialised by the caller.  The call only enqueues work on
 * `stream`. */
#define PTSBE_NOALLOC_SCRATCH_BYTES (64ull << 20)
ptsbe_status ptsbe_run_batch_noalloc(ptsbe_plan_t plan, ptsbe_trajset_t ts, const ptsbe_run_opts* opts,
                                     void* d_bits, uint32_t* d_traj, uint64_t capacity, uint8_t* d_mr_bits,
                                     uint32_t* d_status, void* stream);

/* Captured execution (HIP graph): the same arguments as ptsbe_run_batch.  The
 * tables are uploaded into the workspace now (the call waits for `stream`),
 * then the run's device work -- tile passes, measure-resets, scans, sampler --
 * is captured from `stream` (a created stream, not the default one) and
 * instantiated.  Each ptsbe_graph_launch replays it: same inputs, same
 * outputs, no host work.  The workspace and output buffers must outlive the
 * graph and must not be reused by other calls in between.  opts->timing must
 * be NULL; an empty trajectory set fails with PTSBE_E_ARG. */
typedef struct ptsbe_graph_s* ptsbe_graph_t;
ptsbe_status ptsbe_graph_create(ptsbe_plan_t plan, ptsbe_trajset_t ts, const ptsbe_run_opts* opts,
                                void* d_ws, size_t ws_bytes, void* d_bits, uint32_t* d_traj,
                                uint64_t capacity, uint8_t* d_mr_bits, void* stream,
                                ptsbe_graph_t* out);
ptsbe_status ptsbe_graph_launch(ptsbe_graph_t graph, void* stream);
void ptsbe_graph_destroy(ptsbe_graph_t graph);

/* Inspection: the device tables a run of `ts` would upload (fused passes, ops,
 * slot matrices, per-trajectory overrides, shot and chunk offsets, execution
 * steps), for host-side checks of the fused program.  With out == NULL only
 * *bytes is set.  offsets receives 16 uint64 values: byte offsets of passes,
 * ops, slot defaults, matrix pool, override offsets, overrides, shot offsets,
 * chunk offsets, execution steps, then the counts of passes, ops, slots, pool
 * entries, overrides and execution steps, then the total size. */
ptsbe_status ptsbe_trajset_tables(ptsbe_trajset_t ts, const double* params, uint32_t sort_chunk, void* out,
                                  size_t* bytes, uint64_t* offsets);

/* Inspection of the adjoint gradient's reverse-sweep program: the same table
 * blob and 16 offsets as ptsbe_trajset_tables, with DOT operations (type 10,
 * local pair bit in `a`, generator 1/2/3 = X/Y/Z in `b`, gradient-term index
 * slot[0] | slot[1] << 16).  *n_dot receives the number of gradient terms and
 * dot_param (optional, *n_dot entries) the parameter index of each.
 * PTSBE_E_UNSUPPORTED if the plan has no adjoint program. */
ptsbe_status ptsbe_trajset_adjoint_tables(ptsbe_trajset_t ts, const double* params, void* out,
                                          size_t* bytes, uint64_t* offsets, uint32_t* n_dot,
                                          uint32_t* dot_param);

/* Wait for `stream` and read the device status word of a workspace last used
 * by ptsbe_run_batch: PTSBE_OK or PTSBE_E_NONDET_MEASURE. */
ptsbe_status ptsbe_run_status(ptsbe_plan_t plan, const void* d_ws, void* stream);

/* Distinct shots (Sec. 4, Fig. 4: the fraction of a trajectory's shots that
 * are distinct; its expectation is sum_x 1 - (1 - p_x)^m).  For the shots of
 * ts as ptsbe_run_batch wrote them (d_bits: device, total_shots entries, uint32
 * for n <= 32 qubits, else uint64, trajectory alpha's m_alpha shots contiguous
 * in trajectory order): d_unique (device, n_traj uint64) receives each
 * trajectory's number of distinct basis indices; optionally d_pair_index (same
 * width and length as d_bits) and d_pair_count (device, total_shots uint32)
 * receive, from trajectory alpha's first shot position on, its distinct
 * indices in order of first appearance in its shots with their shot counts
 * (entries past d_unique[alpha] within its range are left untouched).  One
 * open-addressing hash table per trajectory lives in the caller's workspace
 * (256-byte aligned, size from ptsbe_unique_workspace_size: max_batch
 * consecutive trajectories at once, 0 = all); trajectories are processed in the
 * largest batches that fit.  Results do not depend on thread scheduling.
 * Errors: PTSBE_E_ARG (null outputs, misaligned or too small workspace),
 * PTSBE_E_UNSUPPORTED (2^32 or more shots in one trajectory).  The call only
 * enqueues work on `stream`; host staging lives in ts until its next call, so
 * calls on one trajectory set must not overlap. */
ptsbe_status ptsbe_unique_workspace_size(ptsbe_trajset_t ts, uint32_t max_batch, size_t* bytes);
ptsbe_status ptsbe_unique_shots(ptsbe_trajset_t ts, const void* d_bits, void* d_ws, size_t ws_bytes,
                                uint64_t* d_unique, void* d_pair_index, uint32_t* d_pair_count, void* stream);

/* Adjoint gradient of E(theta) = sum_alpha w_alpha <psi_alpha|O|psi_alpha>,
 * w_alpha from ptsbe_trajset_weights (for unitary-mixture noise w does not
 * depend on theta): forward preparation, lambda = O psi, then a reverse sweep that
 * un-applies each operation on psi and lambda and accumulates
 * 2 Re <lambda| dG/dtheta |psi> in FP64 per (trajectory, tile), reduced in a
 * fixed order (deterministic).  O = sum_t coef_t Z-string(zmask_t), 1..64 terms.
 * State-dependent channels (Algorithm 1's state-dependent branch) are decided
 * in the forward preparation exactly as ptsbe_run_batch decides them with the
 * same seed and cfg (Philox stream 4); the state at each decision is
 * checkpointed in the workspace and restored by the reverse sweep, which holds
 * the chosen K_k / sqrt(p_k) fixed: the per-trajectory derivative is then
 * d<phi|O|phi> / <phi|phi> of the unnormalised path state, whose average over
 * paths drawn with their probabilities is the exact derivative (pathwise and
 * score-function terms together).
 * params: host FP64 array of n_params values; d_expval: device, 1 FP64 (E);
 * d_grad: device, n_params FP64.  The workspace (256-byte aligned, size from
 * ptsbe_workspace_size with mode PTSBE_RUN_ADJOINT) is split into batches of
 * trajectories that fit it.  Errors: PTSBE_E_UNSUPPORTED if the plan has no
 * parameters or holds measure-reset / projection steps; PTSBE_E_OOM if not even
 * one trajectory fits the workspace.  The call only enqueues work on `stream`. */
ptsbe_status ptsbe_adjoint_grad(ptsbe_plan_t plan, ptsbe_trajset_t ts, const double* params,
                                const double* obs_coef, const uint64_t* obs_zmask, uint32_t n_terms,
                                uint64_t seed, uint32_t cfg, void* d_ws, size_t ws_bytes,
                                double* d_expval, double* d_grad, void* stream);

/* ---------------------------------------------------------- gate library */

/* Pauli twirl of a channel (nq 1 or 2; n_kraus operators, complex128 row-major
 * interleaved, basis index bit j = the site's j-th qubit): averaging over
 * conjugation by the 4^nq Pauli strings leaves the Pauli channel with
 * probs[P] = sum_k |Tr(P^dag K_k)|^2 / 4^nq (the diagonal of the Pauli transfer
 * matrix); string P has base-4 digit j (0 I, 1 X, 2 Y, 3 Z) on qubit j.  probs
 * holds 4^nq doubles.  Errors: PTSBE_E_ARG (bad sizes), PTSBE_E_NOT_CPTP. */
ptsbe_status ptsbe_pauli_twirl(uint32_t nq, const double* kraus, uint32_t n_kraus, double* probs);

/* Standard gate matrices (complex128, row-major interleaved) for building
 * circuits: name in {U3, RX, RY, RZ, H, X, Y, Z, S, T, CZ, CNOT, SWAP};
 * params as in the usual definitions (U3: theta, phi, lambda).  out holds
 * 2 * 4^nq doubles; *nq receives the qubit count. */
ptsbe_status ptsbe_std_gate(const char* name, const double* params, double* out, uint32_t* nq);
/* Standard channels: name in {depolarizing (nq 1|2, p), xflip (p), pauli (px, py, pz),
 * u3_mixture (p, theta, phi, lambda), amplitude_damping (gamma)}.  out holds
 * n_kraus * 2 * 4^nq doubles; *n_kraus receives the operator count. */
ptsbe_status ptsbe_std_channel(const char* name, uint32_t nq, const double* params, double* out,
                               uint32_t* n_kraus);

#ifdef __cplusplus
}
#endif

#endif /* PTSBE_H */
