// ptsbe_run_batch without allocation: the same batched execution, with its
// workspace (tables, launch routes, the resident batch of states, FP64 scan
// partials, measure-reset partials, the status word) in a fixed device array
// of this library instead of a caller buffer, for callers that cannot allocate
// device memory (code under stream capture, tight serving loops).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "host.hpp"

namespace ptsbe {
ptsbe_status run_batch(const Plan& P, TrajSet& ts, const ptsbe_run_opts* o, void* d_ws, size_t ws_bytes,
                       void* d_bits, uint32_t* d_traj, uint64_t capacity, uint8_t* d_mr_bits, void* stream,
                       hipGraphExec_t* graph_out, bool no_alloc, uint32_t* d_status);
}  // namespace ptsbe

namespace {

constexpr size_t kScratchBytes = size_t(PTSBE_NOALLOC_SCRATCH_BYTES);

// One copy per device, held from the first use of this module until the
// process ends.  Host code never uses this name as an address: the device
// address comes from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
ptsbe_status scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return ptsbe::fail(PTSBE_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return ptsbe::fail(PTSBE_E_DEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return ptsbe::fail(PTSBE_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return PTSBE_OK;
}

}  // namespace

extern "C" ptsbe_status ptsbe_run_batch_noalloc(ptsbe_plan_t plan, ptsbe_trajset_t ts, const ptsbe_run_opts* opts,
                                                void* d_bits, uint32_t* d_traj, uint64_t capacity,
                                                uint8_t* d_mr_bits, uint32_t* d_status, void* stream) {
  try {
    if (!plan || !ts) return ptsbe::fail(PTSBE_E_ARG, "null argument");
    if (ts->ts->plan.get() != plan->plan.get())
      return ptsbe::fail(PTSBE_E_ARG, "trajectory set belongs to another plan");
    void* ws = nullptr;
    ptsbe_status st = scratch_ptr(&ws);
    if (st != PTSBE_OK) return st;
    st = ptsbe::run_batch(*plan->plan, *ts->ts, opts, ws, kScratchBytes, d_bits, d_traj, capacity, d_mr_bits,
                          stream, nullptr, true, d_status);
    if (st == PTSBE_E_OOM)
      return ptsbe::fail(PTSBE_E_OOM, "one trajectory needs more than the " + std::to_string(kScratchBytes >> 20) +
                                          " MiB of the library's fixed device scratch");
    return st;
  } catch (const std::bad_alloc&) {
    return ptsbe::fail(PTSBE_E_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return ptsbe::fail(PTSBE_E_ARG, std::string("internal error: ") + e.what());
  } catch (...) {
    return ptsbe::fail(PTSBE_E_ARG, "internal error");
  }
}
