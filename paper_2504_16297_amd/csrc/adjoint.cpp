// Adjoint gradient of the probability-weighted trajectory ensemble.
#include "host.hpp"

namespace ptsbe {

ptsbe_status adjoint_grad(const Plan& P, TrajSet& ts, const double* params, const double* coef,
                          const uint64_t* zmask, uint32_t n_terms, void* d_ws, size_t ws_bytes, double* d_expval,
                          double* d_grad, void* stream) {
  (void)P; (void)ts; (void)params; (void)coef; (void)zmask; (void)n_terms; (void)d_ws; (void)ws_bytes;
  (void)d_expval; (void)d_grad; (void)stream;
  return fail(PTSBE_E_UNSUPPORTED, "adjoint gradient not built yet");
}

}  // namespace ptsbe
