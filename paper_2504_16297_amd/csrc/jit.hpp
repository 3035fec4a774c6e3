// Pass compiler: each register-layout tile pass of a plan becomes its own
// gfx950 kernel, generated as HIP source from the pass's fixed operation list
// and compiled with hiprtc once per plan.  The trajectory-dependent part of a
// pass (which matrix each slot holds) stays in the device tables, so one
// compiled kernel serves every trajectory of every set run on the plan.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ptsbe.h"
#include "kernels.hpp"

namespace ptsbe {

struct Pass;
struct Plan;

struct JitProgram {
  std::mutex mu;
  bool built = false;
  ptsbe_status build_status = PTSBE_OK;
  std::string build_error;
  std::vector<int> pass_kernel;            // pass -> compiled kernel index, -1 = interpreter kernel
  std::vector<int> adj_pass_kernel;        // reverse-sweep pass -> compiled kernel index, -1 = generic
  std::vector<std::string> names;          // kernel index -> symbol
  std::vector<std::string> sources;        // kernel index -> HIP source
  std::vector<uint32_t> tile_elems;        // kernel index -> amplitudes of LDS tile space
  std::vector<uint32_t> tiles_per_block;   // kernel index -> tiles of a state per workgroup (1 or 2)
  std::vector<std::vector<char>> code;     // kernel index -> code object
  double compile_seconds = 0.0;
  // per device: loaded modules and kernel handles
  std::map<int, std::vector<hipModule_t>> modules;
  std::map<int, std::vector<hipFunction_t>> functions;
};

// HIP source of a register-layout pass kernel named `name`, or "" if the pass
// is outside what the compiler handles (then the interpreter kernel runs it).
// `split`: register changes move through half a tile of LDS in two rounds
// (less LDS per workgroup, more resident workgroups), unless a 4x4 matrix off
// the register bits needs the whole tile.  *tile_elems receives the LDS tile
// size in amplitudes.
// `dual`: the adjoint sweep's kernel (signature (PassArgs, V* lam, double*
// partial, uint32_t n_dot)): every operation acts on psi and lambda, DOT ops
// write one FP64 partial per (trajectory, tile, wavefront, gradient term).
// `swz`: states stored swizzled (kernels.hpp swizzle(); no effect for n <= 12).
// `nt`: state loads and stores of the forward passes with nontemporal hints.
// `waves`: waves per SIMD the kernel's register budget is set for (0 = the
// compiler's choice).
// `tpb`: tiles per workgroup (2: a forward pass of a state larger than one tile
// runs tiles 2b and 2b + 1 in workgroup b, the second tile's loads issued up
// front; the grid's x extent halves); *tiles_per_block receives what was used.
std::string jit_pass_source(const Pass& ps, int n, int precision, const std::string& name, bool split,
                            uint32_t* tile_elems, bool dual = false, int waves = 0, bool swz = true,
                            bool nt = false, int tpb = 1, uint32_t* tiles_per_block = nullptr);

// Generate and compile every pass kernel of the plan (host only, no device
// needed).  Idempotent; thread-safe.
ptsbe_status jit_build(const Plan& P);

// Launch pass `pass` of the plan through its compiled kernel on `stream`
// (loads the code objects on the current device at first use).  `a` carries
// the plan-wide tables; the pass-local slot defaults are selected here.
template <typename V>
hipError_t jit_launch(const Plan& P, uint32_t pass, const PassArgs<V>& a, uint32_t rows, hipStream_t s);

// Load the compiled kernels on the current device now (before stream capture).
hipError_t jit_load(const Plan& P);

// True if the compiled kernels are built and already loaded on the current
// device (no loading, so no device allocation).
bool jit_loaded(const Plan& P);

// True if pass `pass` runs through a compiled kernel.
bool jit_has(const Plan& P, uint32_t pass);

// The reverse-sweep (adjoint) pass `pass` through its compiled kernel: psi in
// a.p.states, lambda in a.lam; gradient partials at
// [(trajectory * tiles * W + tile * W + wavefront) * n_dot + term], W =
// jit_adjoint_waves(k) wavefronts per workgroup.
bool jit_has_adjoint(const Plan& P, uint32_t pass);
template <typename V>
hipError_t jit_adjoint_launch(const Plan& P, uint32_t pass, const AdjArgs<V>& a, uint32_t rows, hipStream_t s);
uint32_t jit_adjoint_waves(uint32_t k);

}  // namespace ptsbe
