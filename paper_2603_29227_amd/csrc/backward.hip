// Query backward (adjoint) — placeholder until the adjoint kernels land.
#include "ksdf_internal.h"

namespace ksdf {

size_t backward_workspace_bytes(const ksdf_model* m, long Q) {
  (void)m;
  (void)Q;
  return 0;
}

int launch_backward(const ksdf_model* m, const void* points, long Q, const int8_t* sign,
                    const void* d_mean, const void* d_grad, const void* d_var,
                    const void* d_var_f, void* d_points, double* d_hyper, void* ws,
                    size_t ws_bytes, hipStream_t s) {
  set_error("backward not available");
  return KSDF_ERR_UNSUPPORTED;
}

}  // namespace ksdf
