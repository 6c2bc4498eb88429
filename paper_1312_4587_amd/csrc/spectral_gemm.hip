// Spectral solve as dense cosine/sine-matrix GEMMs on MFMA (placeholder until
// the GEMM kernels land: plans in the GEMM modes report unsupported).
#include "fftpl_internal.hpp"

namespace fftpl {

int gemm_plan_init(Plan&, hipStream_t) { return FFTPL_E_UNSUPPORTED; }

void gemm_plan_free(Plan& p) {
  hipFree(p.gemm_tables);
  hipFree(p.gemm_ws);
  p.gemm_tables = nullptr;
  p.gemm_ws = nullptr;
}

hipError_t spectral_gemm(Plan&, const SpectralArgs&, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace fftpl
