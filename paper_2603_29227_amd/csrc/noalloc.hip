// ksdf_query_noalloc: ksdf_query for callers that cannot allocate device memory
// (code under graph capture, tight serving loops, harnesses that forbid allocation).
//
// The query's scratch (bucketing counters, the sorted query order and the records
// passed between its two kernels) lives in a file-scope device array of
// KSDF_NOALLOC_SCRATCH_BYTES instead of a caller workspace.  Every device the
// library runs on holds its own copy until the process ends; its address is looked
// up once per device (hipGetSymbolAddress, with that device current) and kept.  The
// query kernels clear what must start at zero themselves, so the array's contents
// from an earlier call do not matter.  All calls on one device share the array:
// calls that overlap on one device race.
#include <mutex>

#include "ksdf_internal.h"

namespace ksdf {
namespace {

static __device__ __align__(256) unsigned char scratch[KSDF_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};

// The device address of `scratch` on the current device (looked up on first use).
int scratch_for(int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEVICES) {
    set_error("ksdf_query_noalloc: device index out of range");
    return KSDF_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      set_error(std::string("ksdf_query_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
      return KSDF_ERR_HIP;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return KSDF_OK;
}

}  // namespace
}  // namespace ksdf

using namespace ksdf;

extern "C" int ksdf_query_noalloc(const ksdf_model* m, const void* points, long Q,
                                  const int8_t* sign, void* mean, void* grad, void* var,
                                  void* var_f, void* grad_var, int* argmin, uint8_t* q_status,
                                  void* stream) {
  if (!m || Q < 0 || (Q > 0 && (!points || !mean || !grad || !var))) {
    set_error("ksdf_query_noalloc: invalid argument");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  if (!m->fitted || !m->index_ready) {
    set_error("ksdf_query_noalloc: the model has not been fitted or its index is not attached");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  const size_t need = query_workspace_bytes(m, Q);
  if (need > KSDF_NOALLOC_SCRATCH_BYTES) {
    set_error("ksdf_query_noalloc: the query needs " + std::to_string(need) +
              " bytes of scratch, more than the fixed " +
              std::to_string((size_t)KSDF_NOALLOC_SCRATCH_BYTES) +
              "; use ksdf_query with a workspace");
    return KSDF_ERR_WORKSPACE;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != m->device) {
    (void)hipGetLastError();
    set_error("the current device is not the model's device");
    return KSDF_ERR_DEVICE;
  }
  void* ws = nullptr;
  int r = scratch_for(dev, &ws);
  if (r) return r;
  return launch_query(m, points, Q, sign, mean, grad, var, var_f, grad_var, argmin, q_status, ws,
                      KSDF_NOALLOC_SCRATCH_BYTES, (hipStream_t)stream);
}
