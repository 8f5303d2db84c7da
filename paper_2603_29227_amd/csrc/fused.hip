// Persistent fused fit + query launch (FP32 models, cells with uneven m).
//
// One launch of resident workgroups (256 threads) drains a task queue:
//   tasks [0, n_fit)            fit one cell with the whole workgroup, largest m first
//                               (fit32_cell of the cell's m bucket, FP64 refit in place
//                               when the condition estimate asks for it);
//   tasks [n_fit, n_fit + n_q)  4 query tiles of 64 bucketed queries, one per wave.
// Every fit task is dequeued before any query task, so a workgroup that holds a query
// task waits (acquire) only for fit tasks that other running workgroups already hold:
// the wait always ends.  No query reads cell data before every fit has released its
// writes, so no cache can hold a stale copy of them.  The spin is bounded (a per-model
// limit, settable for tests); on expiry the workgroup stops waiting, every query it
// then answers carries KSDF_Q_FIT_TIMEOUT, and the model's flag in its store records
// the expiry for ksdf_model_check.
#include "fit_dev.h"
#include "query_dev.h"

namespace ksdf {
namespace {

constexpr int FT = 256;
constexpr int WAVES = FT / 64;

struct FusedCtl {
  int* next;          // task counter
  int* done;          // fit tasks completed
  int* timeout;       // the model's flag (store-resident): set when a wait expired
  const int* order;   // cells in fit order (m descending)
  int n_fit;
  long n_qtasks;
  long spin_limit;    // sleeps before a wait gives up
};

// Fit tasks and query tiles run in two consecutive loops (a workgroup's first query
// task ends its fit loop), so values that the compiler keeps live across one loop are
// not live in the other and the kernel needs the registers of the larger part, not of
// both.
template <int MB>
__device__ __forceinline__ bool fit32_task(const FitArgs& F, int c, float* smem) {
  return fit32_cell<MB>(F, c, smem);
}

template <int KM, int MB, int MF>
__global__ void __launch_bounds__(FT) fused_kernel(FitArgs F, FastArgs Q, FusedCtl C) {
  extern __shared__ float smem[];
  __shared__ long task_sh;
  const long n_total = C.n_fit + C.n_qtasks;
  auto grab = [&]() -> long {
    __syncthreads();
    if (threadIdx.x == 0) task_sh = atomicAdd(C.next, 1);
    __syncthreads();
    return task_sh;
  };
  long t = grab();
  while (t < C.n_fit) {
    const int c = C.order[t];
    const int m = F.offsets[c + 1] - F.offsets[c];
    bool need64;
    if (m <= 16) {
      need64 = fit32_task<16>(F, c, smem);
    } else if (m <= 32 || MF <= 32) {
      need64 = fit32_task<32>(F, c, smem);
    } else if (m <= 64 || MF <= 64) {
      if constexpr (MF >= 64) need64 = fit32_task<64>(F, c, smem);
      else need64 = true;
    } else {
      if constexpr (MF >= 128) need64 = fit32_task<128>(F, c, smem);
      else need64 = true;
    }
    if (need64) fit64_cell(F, c, reinterpret_cast<double*>(smem));
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(C.done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    t = grab();
  }
  if (t >= n_total) return;
  // every fit task has been taken: wait until they have all been released
  __shared__ int expired_sh;
  if (threadIdx.x == 0) {
    long spins = 0;
    int expired = 0;
    while (__hip_atomic_load(C.done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < C.n_fit) {
      if (spins >= C.spin_limit) {
        expired = 1;
        atomicOr(C.timeout, 1);
        break;
      }
      __builtin_amdgcn_s_sleep(8);
      ++spins;
    }
    expired_sh = expired;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const bool expired = expired_sh != 0;
  const int wave = threadIdx.x / 64;
  do {
    const long sq = ((t - C.n_fit) * WAVES + wave) * 64 + (threadIdx.x & 63);
    Pass1 p1 = query_pass1<KM>(Q, sq);
    if (expired) p1.flags |= PASS1_FIT_TIMEOUT;   // the cells it read may be unreleased
    query_finish_t<MB, false, false, false>(Q, p1);   // the fused launch serves RBF models
    t = grab();
  } while (t < n_total);
}

__global__ void fused_reset_kernel(int* ctl) {
  if (threadIdx.x < 2) ctl[threadIdx.x] = 0;
}

template <int KM, int MB, int MF>
int launch_fused_t(ksdf_model* m, FitArgs& F, FastArgs& A, FusedCtl& C, hipStream_t s) {
  const size_t smem = std::max(fit32_smem_floats<MF>() * sizeof(float),
                               FIT64_SMEM_DOUBLES * sizeof(double));
  auto kern = fused_kernel<KM, MB, MF>;
  // attribute and occupancy are taken once per kernel, so that a launch made under
  // stream capture issues no device-attribute calls
  static int per_cu = -1;
  if (per_cu < 0) {
    KSDF_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    int occ = 0;
    KSDF_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, FT, smem));
    per_cu = std::max(occ, 1);
  }
  const int cus = std::max(m->n_cu, 1);
  const long tasks = C.n_fit + C.n_qtasks;
  long grid = (long)per_cu * cus;
  if (grid > tasks) grid = tasks;
  if (grid < 1) grid = 1;
  timer_mark(m, KSDF_TIMER_FUSED, 0, s);
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(FT), smem, s, F, A, C);
  launch_linv(m, s);
  timer_mark(m, KSDF_TIMER_FUSED, 1, s);
  KSDF_HIP_TRY(hipGetLastError());
  return KSDF_OK;
}

}  // namespace

size_t fused_workspace_bytes(const ksdf_model* m, long Q) {
  return query_fast_workspace_bytes(m, Q) + 256;
}

int launch_fit_query_fused(ksdf_model* m, const void* pts, int dtype, const void* svar,
                           uint8_t* cell_status, const void* points, long Q, const int8_t* sign,
                           void* mean, void* grad, void* var, void* var_f, void* grad_var, int* argmin,
                           uint8_t* q_status, void* ws, size_t ws_bytes, hipStream_t s) {
  (void)ws_bytes;
  FitArgs F = make_fit_args(m, pts, dtype, svar, cell_status);
  F.emit32 = 1;
  F.list = nullptr;
  FastArgs A = make_fast_args(m, points, Q, sign, mean, grad, var, var_f, grad_var, argmin, q_status);
  int* ctl = reinterpret_cast<int*>(static_cast<char*>(ws) + query_fast_workspace_bytes(m, Q));
  hipLaunchKernelGGL(fused_reset_kernel, dim3(1), dim3(64), 0, s, ctl);
  if (Q > 0) {
    int r = launch_bucketing(m, A, ws, s);
    if (r != KSDF_OK) return r;
  }
  FusedCtl C{};
  C.next = ctl;
  C.done = ctl + 1;
  C.timeout = m->flags;
  C.spin_limit = m->wait_limit;
  C.order = m->fused_order;
  C.n_fit = m->n_cells;
  C.n_qtasks = (Q + FT - 1) / FT;
  if (C.n_fit + C.n_qtasks == 0) return KSDF_OK;
  const bool k8 = m->k_fuse <= 8;
  const int mf = m->max_m <= 16 ? 16 : m->max_m <= 32 ? 32 : m->max_m <= 64 ? 64 : 128;
  if (k8) {
    if (mf <= 32) return launch_fused_t<8, 64, 32>(m, F, A, C, s);
    if (mf == 64) return launch_fused_t<8, 64, 64>(m, F, A, C, s);
    return launch_fused_t<8, 128, 128>(m, F, A, C, s);
  }
  if (mf <= 32) return launch_fused_t<16, 64, 32>(m, F, A, C, s);
  if (mf == 64) return launch_fused_t<16, 64, 64>(m, F, A, C, s);
  return launch_fused_t<16, 128, 128>(m, F, A, C, s);
}

}  // namespace ksdf
