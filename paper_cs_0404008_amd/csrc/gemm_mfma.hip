// Matrix-core (MFMA) kernels for the exact matrix product: placeholder until
// the FP64 and int8 paths land; every call falls through to the exact
// vector-ALU kernel.
#include "fdot_internal.h"

fdot_status_t fd_launch_gemm_mfma(const fdot_field_s*, size_t, size_t, size_t, const void*, size_t,
                                  const void*, size_t, void*, size_t, hipStream_t, bool* handled) {
  *handled = false;
  return FDOT_E_UNSUPPORTED;
}
