// Per-cell log-GP fit (Sec. IV-B.1, eq. log_gp_posterior_mean; RBF of Table I).
//
// One workgroup per cell (256 threads, 4 waves of 64).  The workgroup gathers the
// cell's samples into cell-local coordinates, assembles A = K + Sigma, factors it
// A = L L^T in place (right-looking, packed lower triangle), solves a = A^{-1} 1
// with wave-0 triangular solves whose dot products reduce by cross-lane shuffles,
// and writes the per-cell store: (p_i, a_i), sigma_i^2, the packed factor with the
// reciprocal diagonal, the sample bounding box and A+ = sum of positive a_i.
//
// FP32 cells keep A in LDS (float-float entries plus the FP32 factor, 99 KB at
// m = 128) and estimate cond_2(A) by power and inverse iteration; a cell above the
// threshold or with a non-positive pivot is queued for the FP64 kernel, which
// factors in global memory (the plain FP64 path uses that kernel for every cell).
#include "fit_dev.h"

namespace ksdf {
namespace {

constexpr int FIT_THREADS = 256;

template <int MB>
__global__ void __launch_bounds__(FIT_THREADS) fit32_kernel(FitArgs A, const int* list) {
  __shared__ float smem[fit32_smem_floats<MB>()];
  const int c = list[blockIdx.x];
  const bool need64 = fit32_cell<MB>(A, c, smem);
  if (threadIdx.x == 0 && need64) {
    const int slot = atomicAdd(A.fb_count, 1);
    A.fb_list[slot] = c;
  }
}

__global__ void set_int_kernel(int* p, int v) { *p = v; }

__global__ void __launch_bounds__(FIT_THREADS) fit64_kernel(FitArgs A) {
  __shared__ double smem[FIT64_SMEM_DOUBLES];
  const int count = A.list ? *A.list_count : A.n_cells;
  for (int t = blockIdx.x; t < count; t += gridDim.x) fit64_cell(A, A.list ? A.list[t] : t, smem);
}

}  // namespace

int launch_fit(ksdf_model* m, const void* pts, int dtype, const void* svar, uint8_t* user_status,
               hipStream_t s) {
  FitArgs A = make_fit_args(m, pts, dtype, svar, user_status);
  if (m->n_cells == 0) return KSDF_OK;
  if (m->precision == KSDF_FP64) {
    A.list = nullptr;
    A.emit32 = 0;
    timer_mark(m, KSDF_TIMER_FIT, 0, s);
    hipLaunchKernelGGL(fit64_kernel, dim3(m->n_cells), dim3(FIT_THREADS), 0, s, A);
    timer_mark(m, KSDF_TIMER_FIT, 1, s);
  } else {
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, s, m->fb_count, 0);
    timer_mark(m, KSDF_TIMER_FIT, 0, s);
    // m buckets: cells below the tuned smallest bucket merge into it
    const int* lists = m->bucket_cells;
    const int* bs = m->bucket_start;
    const int minb = m->tuning.fit_min_bucket;
    const int lo32 = minb >= 32 ? bs[0] : bs[1];
    const int lo64 = minb >= 64 ? bs[0] : bs[2];
    if (minb < 32 && bs[1] > bs[0])
      hipLaunchKernelGGL(fit32_kernel<16>, dim3(bs[1] - bs[0]), dim3(FIT_THREADS), 0, s, A, lists + bs[0]);
    if (minb < 64 && bs[2] > lo32)
      hipLaunchKernelGGL(fit32_kernel<32>, dim3(bs[2] - lo32), dim3(FIT_THREADS), 0, s, A, lists + lo32);
    if (bs[3] > lo64)
      hipLaunchKernelGGL(fit32_kernel<64>, dim3(bs[3] - lo64), dim3(FIT_THREADS), 0, s, A, lists + lo64);
    if (bs[4] > bs[3])
      hipLaunchKernelGGL(fit32_kernel<128>, dim3(bs[4] - bs[3]), dim3(FIT_THREADS), 0, s, A, lists + bs[3]);
    A.list = m->fb_list;
    A.list_count = m->fb_count;
    A.emit32 = 1;
    const int grid = m->n_cells < 2048 ? m->n_cells : 2048;
    hipLaunchKernelGGL(fit64_kernel, dim3(grid), dim3(FIT_THREADS), 0, s, A);
    timer_mark(m, KSDF_TIMER_FIT, 1, s);
  }
  KSDF_HIP_TRY(hipGetLastError());
  return KSDF_OK;
}

}  // namespace ksdf
