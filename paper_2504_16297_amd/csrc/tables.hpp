// Device-visible tables of a PTSBE run: the fused tile passes of the plan,
// their matrix slots, and each trajectory's per-pass overrides.  Built on the
// host once per (plan, trajectory set, parameters) and copied into the head
// of the caller's workspace with one transfer.
#pragma once

#include <stdint.h>

namespace ptsbe {

constexpr int kMaxTileBits = 13;
constexpr int kMaxQubits = 35;  // 2^35 complex64 = 256 GiB: one trajectory on one 288 GB GPU

// Fused operation types inside a tile pass.
enum DOpType : uint8_t {
  DOP_M1 = 1,     // 2x2 matrix on local bit a
  DOP_M2 = 2,     // 4x4 matrix on local bits (a = matrix bit 0, b = matrix bit 1)
  DOP_D1 = 3,     // diagonal (2 entries) on global qubit ga
  DOP_D2 = 4,     // diagonal (4 entries) on global qubits (ga = matrix bit 0, gb = bit 1)
  DOP_MR = 5,     // measure-reset apply on local bit a: |0><b| / sqrt(p_b), b from the device record
  DOP_DSIGN = 6,  // +-1 diagonal on (ga, gb): negate where bit (ba + 2 bb) of `slot` is set;
                  // a / b are the local bits of ga / gb or 255 (b = 254: one-qubit sign on ga)
  DOP_PHASE = 7,  // register kernel: new set of 4 register bits (a, b, ga, gb), via an LDS transpose
  DOP_M1G = 8,    // register kernel: 2x2 matrix slot[j] on register position j = 0..3 (the
                  // ascending register bits); `mask` marks the non-identity positions
  DOP_SFLIP = 9,  // register kernel: apply the signs accumulated by the preceding DOP_DSIGNs
  DOP_KR = 11,    // state-dependent channel on local bit a: K_k / sqrt(p_k) with k and the factor from
                  // the device record entry slot[0]; the Kraus operators (4 entries each) at slot slot[1]
  DOP_DOT = 10,   // adjoint kernel: partial Im<lambda|P_a|psi> of gradient term slot[0] | slot[1] << 16,
                  // P = X/Y/Z by b = 1/2/3 on local bit a
};

constexpr uint32_t kRegBits = 4;      // amplitudes per thread = 2^kRegBits in the register kernel
constexpr uint32_t kMinRegTile = 6;   // smallest tile run by the register kernel (one wavefront)

struct DOp {             // 16 bytes: four 32-bit words
  uint8_t type;
  uint8_t a, b;        // local tile bits (M1, M2, MR); for D1/D2 the local bit of ga/gb or 255
  uint8_t ga, gb;      // global qubits (D1, D2)
  uint8_t mask;        // M1G: register positions present
  uint8_t pad0, pad1;
  uint16_t slot[4];    // slot[0]: matrix slot (M1, M2, D1, D2), sign mask (DSIGN), record index
                       // (MR); M1G: slot of register position j
};
static_assert(sizeof(DOp) == 16, "DOp layout");

enum DPassFlags : uint32_t {
  PASS_INIT_ZERO = 1,  // the tile starts from |0...0> instead of being loaded
};

struct DPass {
  uint32_t k;          // tile bits
  uint32_t n_ops;
  uint32_t op_begin;   // index into the DOp array
  uint32_t slot_begin; // index into the slot-default array
  uint32_t n_slots;
  uint32_t flags;
  uint8_t tq[16];      // local bit j -> global qubit (ascending)
  uint8_t oq[48];      // other qubits, ascending (n - k entries)
};

struct DOverride {
  uint32_t slot;       // slot index within the pass
  uint32_t off;        // matrix offset in the pool (complex elements)
};

// Execution step as recorded in the tables (read by the host and by
// inspection tools, not by kernels): a tile pass, or a group of measure-resets.
struct DExec {
  uint32_t pass;       // pass index, or 0xffffffff for a measurement step
  uint32_t nq;         // measurement: number of qubits
  uint32_t q[16];
  uint32_t idx[16];    // measurement: record indices
};

// Offsets (bytes) of each table inside the uploaded block.
struct TableLayout {
  uint64_t passes, ops, slot_default, pool, ov_off, ov, shot_off, chunk_off, exec;
  uint64_t n_passes, n_ops, n_slots, n_pool, n_ov, n_exec;
  uint64_t total;
};

}  // namespace ptsbe
