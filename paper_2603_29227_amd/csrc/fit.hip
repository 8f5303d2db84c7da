// Per-cell log-GP fit (Sec. IV-B.1, eq. log_gp_posterior_mean; RBF of Table I).
//
// Cells with m <= 64 are fitted by one wave each (fit_wave.h: rows in registers, four
// cells per workgroup, no workgroup barriers); larger cells by one workgroup each
// (256 threads, 4 waves of 64), which gathers the cell's samples into cell-local
// coordinates, assembles A = K + Sigma, factors it A = L L^T in place (right-looking,
// packed lower triangle), solves a = A^{-1} 1 with wave-0 triangular solves whose dot
// products reduce by cross-lane shuffles.  Both write the per-cell store: (p_i, a_i),
// sigma_i^2, the packed factor with the reciprocal diagonal, the sample bounding box
// and A+ = sum of positive a_i.
//
// The workgroup fit keeps A in LDS (float-float entries plus the FP32 factor, 99 KB
// at m = 128).  Both estimate cond_2(A) by power and inverse iteration; a cell above
// the threshold or with a non-positive pivot is queued for the FP64 kernel, which
// factors in global memory (the plain FP64 path uses that kernel for every cell).
#include <algorithm>

#include "fit_dev.h"
#include "fit_wave.h"
#include "fit_quad.h"

namespace ksdf {
namespace {

constexpr int FIT_THREADS = 256;

// list: the cells to fit; count (device, or null for the grid size): how many of them
template <int MB>
__global__ void __launch_bounds__(FIT_THREADS) fit32_kernel(FitArgs A, const int* list,
                                                            const int* count) {
  __shared__ float smem[fit32_smem_floats<MB>()];
  if (count && (int)blockIdx.x >= *count) return;
  const int c = list[blockIdx.x];
  const bool need64 = fit32_cell<MB>(A, c, smem);
  if (threadIdx.x == 0 && need64) {
    const int slot = atomicAdd(A.fb_count, 1);
    A.fb_list[slot] = c;
  }
}

// One wave per cell for m <= MB <= 64 (fit_wave.h), four cells per workgroup; n: the
// list's length when count is null
template <int MB, bool MATERN>
__global__ void __launch_bounds__(FIT_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
fit32w_kernel(FitArgs A, const int* list,
                                                             const int* count, int n) {
  __shared__ WaveFitLds<MB> lds[FIT_THREADS / 64];
  const int w = threadIdx.x / 64;
  const int t = blockIdx.x * (FIT_THREADS / 64) + w;
  if (t >= (count ? *count : n)) return;
  const int c = list[t];
  const bool need64 = fit32_wave<MB, MATERN>(A, c, lds[w]);
  if ((threadIdx.x & 63) == 0 && need64) {
    const int slot = atomicAdd(A.fb_count, 1);
    A.fb_list[slot] = c;
  }
}

// One workgroup (four waves) per cell for 64 < m <= 128 (fit_quad.h)
template <bool MATERN>
__global__ void __launch_bounds__(FIT_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
fit32q_kernel(FitArgs A, const int* list, const int* count) {
  __shared__ QuadFitLds lds;
  if (count && (int)blockIdx.x >= *count) return;
  const int c = list[blockIdx.x];
  const bool need64 = fit32_quad<MATERN>(A, c, lds);
  if (threadIdx.x == 0 && need64) {
    const int slot = atomicAdd(A.fb_count, 1);
    A.fb_list[slot] = c;
  }
}

// launch a bucket: the one-wave fit up to m = 64, the four-wave fit above
template <int MB>
void launch_bucket(const FitArgs& A, const int* list, const int* count, int n, hipStream_t s) {
  if (n <= 0) return;
  if constexpr (MB <= 64) {
    const int per = FIT_THREADS / 64;
    const dim3 grid((unsigned)((n + per - 1) / per));
    if (A.kernel == KSDF_KERNEL_MATERN32)
      hipLaunchKernelGGL((fit32w_kernel<MB, true>), grid, dim3(FIT_THREADS), 0, s, A, list, count, n);
    else
      hipLaunchKernelGGL((fit32w_kernel<MB, false>), grid, dim3(FIT_THREADS), 0, s, A, list, count, n);
  } else {
    if (A.kernel == KSDF_KERNEL_MATERN32)
      hipLaunchKernelGGL((fit32q_kernel<true>), dim3((unsigned)n), dim3(FIT_THREADS), 0, s, A, list, count);
    else
      hipLaunchKernelGGL((fit32q_kernel<false>), dim3((unsigned)n), dim3(FIT_THREADS), 0, s, A, list, count);
  }
}

__global__ void set_int_kernel(int* p, int v) { *p = v; }

__global__ void __launch_bounds__(FIT_THREADS) fit64_kernel(FitArgs A) {
  __shared__ double smem[FIT64_SMEM_DOUBLES];
  const int count = A.list ? *A.list_count : A.n_cells;
  for (int t = blockIdx.x; t < count; t += gridDim.x) fit64_cell(A, A.list ? A.list[t] : t, smem);
}

// ---- streaming refit (Sec. IV-C, App. G) ----

// Training-queue score of App. G, s = c2 (1 + eta c0), in FP32 with every rounding
// explicit (no contraction), so that a host computation in the same order agrees.
__device__ __forceinline__ float refit_score(const float* dirty, const float* qcount, float eta,
                                             int c) {
  return __fmul_rn(dirty[c], __fadd_rn(1.f, __fmul_rn(eta, qcount[c])));
}

// The dirty cells (c2 > 0) and their scores, appended in any order (wave-aggregated
// slots); n_dirty counts them.  The ranking below does not depend on the order.
__global__ void __launch_bounds__(256) refit_compact_kernel(const float* dirty, const float* qcount,
                                                            float eta, int n, int* dlist,
                                                            float* dscore, int* n_dirty) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const bool mine = i < n && dirty[i] > 0.f;
  const unsigned long long live = __ballot(mine);
  if (!live) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)live) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(n_dirty, __popcll(live));
  base = __shfl(base, leader, 64);
  if (mine) {
    const int slot = base + __popcll(live & ((1ull << lane) - 1ull));
    dlist[slot] = i;
    dscore[slot] = refit_score(dirty, qcount, eta, i);
  }
}

// Rank of every dirty cell by descending score, ties to the lower id, by comparison
// with the other dirty cells through LDS tiles (work grows with the square of the
// dirty count, not of the cell count); the first `budget` ranks name the cells to
// refit.  Launched with one thread per cell: blocks past the dirty count exit.
__global__ void __launch_bounds__(256) refit_rank_kernel(const int* dlist, const float* dscore,
                                                         const int* n_dirty, int budget, int* sel) {
  __shared__ float ts[256];
  __shared__ int tid_[256];
  const int d = *n_dirty;
  if ((int)blockIdx.x * 256 >= d) return;   // uniform over the block
  const int t = blockIdx.x * 256 + threadIdx.x;
  const bool mine = t < d;
  const float si = mine ? dscore[t] : 0.f;
  const int ci = mine ? dlist[t] : 0;
  int rank = 0;
  for (int base = 0; base < d; base += 256) {
    __syncthreads();
    const int j = base + threadIdx.x;
    ts[threadIdx.x] = j < d ? dscore[j] : 0.f;
    tid_[threadIdx.x] = j < d ? dlist[j] : 0;
    __syncthreads();
    const int lim = min(256, d - base);
    for (int k = 0; k < lim; ++k) {
      const float sj = ts[k];
      rank += (sj > si || (sj == si && tid_[k] < ci)) ? 1 : 0;
    }
  }
  if (mine && rank < budget) sel[rank] = ci;
}

// n_sel = min(budget, n_dirty); clears the per-bucket counts
__global__ void refit_count_kernel(const int* n_dirty, int budget, int* n_sel, int* bcount) {
  if (threadIdx.x == 0) *n_sel = min(budget, *n_dirty);
  if (threadIdx.x < 4) bcount[threadIdx.x] = 0;
}

// the selected cells into per-m-bucket lists (the bucket sizing of the full fit)
__global__ void __launch_bounds__(256) refit_bucket_kernel(const int* sel, const int* n_sel,
                                                           const int* offsets, int minb, int budget,
                                                           int* blist, int* bcount) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= *n_sel) return;
  const int c = sel[i];
  const int mc = offsets[c + 1] - offsets[c];
  int bk = mc <= 16 ? 0 : mc <= 32 ? 1 : mc <= 64 ? 2 : 3;
  if (minb >= 32 && bk < 1) bk = 1;
  if (minb >= 64 && bk < 2) bk = 2;
  const int pos = atomicAdd(&bcount[bk], 1);
  blist[(long)bk * budget + pos] = c;
}

// after the refit: c2 = 0 and c0 halved for the refitted cells (App. G)
__global__ void __launch_bounds__(256) refit_reset_kernel(const int* sel, const int* n_sel,
                                                          float* dirty, float* qcount) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= *n_sel) return;
  const int c = sel[i];
  dirty[c] = 0.f;
  qcount[c] = 0.5f * qcount[c];
}

// Query counters of App. G in two steps, so that the result does not depend on the
// order of the atomics: an integer histogram of the argmin cells (one atomic per
// distinct cell of a wave; queries that arrive spatially ordered mostly share their
// argmin cell within a wave), then one addition per cell, c0 = min(c0 + count, cap),
// rounded once.  (Halving on refit leaves c0 fractional, so float atomics adding
// counts to it directly would round differently in different orders.)  Argmins
// outside [0, n_cells) are not counted.
__global__ void __launch_bounds__(256) zero_kernel(unsigned* h, int n) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c < n) h[c] = 0u;
}

__global__ void __launch_bounds__(256) count_queries_kernel(const int* argmin, long Q, int n_cells,
                                                            unsigned* hist) {
  const long q = (long)blockIdx.x * 256 + threadIdx.x;
  int c = q < Q ? argmin[q] : -1;
  if (c >= n_cells) c = -1;
  const int lane = threadIdx.x & 63;
  unsigned long long todo = __ballot(c >= 0);
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int key = __shfl(c, leader, 64);
    const unsigned long long same = __ballot(c == key) & todo;
    if (lane == leader) atomicAdd(hist + key, (unsigned)__popcll(same));
    todo &= ~same;
  }
}

// The same counts through a histogram in LDS when the cells fit there: each block
// counts one contiguous range of the queries (neighbouring queries mostly share their
// argmin cell) and adds its non-zero bins to the global histogram, so the global
// atomics fall from one per run of equal argmins to one per (block, cell).
constexpr int CQ_T = 1024;
constexpr int CQ_LDS_CELLS = 16384;
__global__ void __launch_bounds__(CQ_T) count_queries_lds_kernel(const int* argmin, long Q,
                                                                int n_cells, unsigned* hist) {
  __shared__ unsigned h[CQ_LDS_CELLS];
  for (int c = threadIdx.x; c < n_cells; c += CQ_T) h[c] = 0u;
  __syncthreads();
  const long per = (Q + gridDim.x - 1) / gridDim.x;
  const long q0 = (long)blockIdx.x * per;
  const long q1 = q0 + per < Q ? q0 + per : Q;
  for (long q = q0 + threadIdx.x; q < q1; q += CQ_T) {
    const int c = argmin[q];
    if (c >= 0 && c < n_cells) atomicAdd(h + c, 1u);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n_cells; c += CQ_T)
    if (h[c]) atomicAdd(hist + c, h[c]);
}

__global__ void __launch_bounds__(256) count_apply_kernel(const unsigned* hist, float* qcount, int n,
                                                          float cap) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c < n) qcount[c] = fminf(qcount[c] + (float)hist[c], cap);
}

// Dense L^{-1} of each cell (64 x 64, column-major, zero beyond m) from the packed
// factor rows with reciprocal diagonal: lane j solves L x = e_j by forward
// substitution, x_i = -(sum_{k<i} L_ik x_k) / L_ii (x_k = 0 for k < j), x_j = 1 / L_jj,
// with its column in registers and the factor rows read once per wave (uniform
// loads); each lane stores its column as 16-byte pieces (no LDS, so that occupancy
// is set by the registers alone).
__global__ void __launch_bounds__(64) linv_kernel(const int* offsets, const long* loff,
                                                  const float* L, float* Linv) {
  const int c = blockIdx.x, j = threadIdx.x;
  const int m = offsets[c + 1] - offsets[c];
  const float* Lc = L + loff[c];
  float x[64];
#pragma unroll
  for (int i = 0; i < 64; ++i) {
    float xi = 0.f;
    if (i < m) {
      const float* row = Lc + i * (i + 1) / 2;
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
      for (int k = 0; k + 3 < i; k += 4) {
        a0 = fmaf(row[k], x[k], a0);
        a1 = fmaf(row[k + 1], x[k + 1], a1);
        a2 = fmaf(row[k + 2], x[k + 2], a2);
        a3 = fmaf(row[k + 3], x[k + 3], a3);
      }
#pragma unroll
      for (int k = i & ~3; k < i; ++k) a0 = fmaf(row[k], x[k], a0);
      const float r = row[i];
      xi = j == i ? r : (j < i ? -((a0 + a1) + (a2 + a3)) * r : 0.f);
    }
    x[i] = xi;
  }
  float4* out = reinterpret_cast<float4*>(Linv + (long)c * 4096 + (long)j * 64);
#pragma unroll
  for (int i = 0; i < 16; ++i) out[i] = make_float4(x[4 * i], x[4 * i + 1], x[4 * i + 2], x[4 * i + 3]);
}

}  // namespace

void launch_linv(const ksdf_model* m, hipStream_t s) {
  m->linv_ok = false;
  if (!m->Linv32 || !m->tuning.query_mfma || m->n_cells == 0) return;
  hipLaunchKernelGGL(linv_kernel, dim3((unsigned)m->n_cells), dim3(64), 0, s, m->offsets, m->loff,
                     m->L32, m->Linv32);
  m->linv_ok = true;
}

size_t refit_workspace_bytes(const ksdf_model* m, int budget) {
  const long b = std::min(budget, m->n_cells);
  // bucket lists, bucket counts + n_dirty, then the dirty cells' ids and scores
  return 4 * b * sizeof(int) + 8 * sizeof(int) + 2 * (long)m->n_cells * sizeof(int);
}

int launch_refit(ksdf_model* m, const void* pts, int dtype, const void* svar, float* dirty,
                 float* qcount, double eta, int budget, int* sel, int* n_sel, uint8_t* user_status,
                 void* ws, hipStream_t s) {
  if (m->n_cells == 0) {
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, s, n_sel, 0);
    KSDF_HIP_TRY(hipGetLastError());
    return KSDF_OK;
  }
  budget = std::min(budget, m->n_cells);
  int* blist = static_cast<int*>(ws);
  int* bcount = blist + 4L * budget;
  int* n_dirty = bcount + 4;
  int* dlist = bcount + 8;
  float* dscore = reinterpret_cast<float*>(dlist + m->n_cells);
  const unsigned gc = (unsigned)((m->n_cells + 255) / 256);
  const unsigned gb = (unsigned)((budget + 255) / 256);
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, s, n_dirty, 0);
  hipLaunchKernelGGL(refit_compact_kernel, dim3(gc), dim3(256), 0, s, dirty, qcount, (float)eta,
                     m->n_cells, dlist, dscore, n_dirty);
  hipLaunchKernelGGL(refit_rank_kernel, dim3(gc), dim3(256), 0, s, dlist, dscore, n_dirty, budget, sel);
  hipLaunchKernelGGL(refit_count_kernel, dim3(1), dim3(64), 0, s, n_dirty, budget, n_sel, bcount);
  FitArgs A = make_fit_args(m, pts, dtype, svar, user_status);
  timer_mark(m, KSDF_TIMER_FIT, 0, s);
  if (m->precision == KSDF_FP64) {
    A.list = sel;
    A.list_count = n_sel;
    A.emit32 = 0;
    hipLaunchKernelGGL(fit64_kernel, dim3((unsigned)budget), dim3(FIT_THREADS), 0, s, A);
  } else {
    const int minb = m->tuning.fit_min_bucket;
    hipLaunchKernelGGL(refit_bucket_kernel, dim3(gb), dim3(256), 0, s, sel, n_sel, m->offsets, minb,
                       budget, blist, bcount);
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, s, m->fb_count, 0);
    // grid per bucket: at most the budget and at most the cells of that bucket
    const int* bs = m->bucket_start;
    const int lo32 = minb >= 32 ? bs[0] : bs[1];
    const int lo64 = minb >= 64 ? bs[0] : bs[2];
    const int n16 = minb < 32 ? bs[1] - bs[0] : 0;
    const int n32 = minb < 64 ? bs[2] - lo32 : 0;
    const int n64 = bs[3] - lo64, n128 = bs[4] - bs[3];
    launch_bucket<16>(A, blist, bcount, std::min(n16, budget), s);
    launch_bucket<32>(A, blist + budget, bcount + 1, std::min(n32, budget), s);
    launch_bucket<64>(A, blist + 2L * budget, bcount + 2, std::min(n64, budget), s);
    launch_bucket<128>(A, blist + 3L * budget, bcount + 3, std::min(n128, budget), s);
    A.list = m->fb_list;
    A.list_count = m->fb_count;
    A.emit32 = 1;
    hipLaunchKernelGGL(fit64_kernel, dim3((unsigned)std::min(budget, 2048)), dim3(FIT_THREADS), 0, s,
                       A);
  }
  if (m->precision != KSDF_FP64) launch_linv(m, s);
  timer_mark(m, KSDF_TIMER_FIT, 1, s);
  hipLaunchKernelGGL(refit_reset_kernel, dim3(gb), dim3(256), 0, s, sel, n_sel, dirty, qcount);
  KSDF_HIP_TRY(hipGetLastError());
  return KSDF_OK;
}

size_t count_queries_workspace_bytes(const ksdf_model* m) {
  return (size_t)std::max(m->n_cells, 1) * sizeof(unsigned);
}

int launch_count_queries(const ksdf_model* m, const int* argmin, long Q, float* qcount, float cap,
                         void* ws, hipStream_t s) {
  const int n = m->n_cells;
  if (n == 0) return KSDF_OK;
  unsigned* hist = static_cast<unsigned*>(ws);
  const unsigned gc = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(zero_kernel, dim3(gc), dim3(256), 0, s, hist, n);
  if (Q > 0 && n <= CQ_LDS_CELLS) {
    const long blocks = std::min<long>(1024, (Q + CQ_T - 1) / CQ_T);
    hipLaunchKernelGGL(count_queries_lds_kernel, dim3((unsigned)blocks), dim3(CQ_T), 0, s, argmin, Q,
                       n, hist);
  } else if (Q > 0) {
    hipLaunchKernelGGL(count_queries_kernel, dim3((unsigned)((Q + 255) / 256)), dim3(256), 0, s,
                       argmin, Q, n, hist);
  }
  hipLaunchKernelGGL(count_apply_kernel, dim3(gc), dim3(256), 0, s, hist, qcount, n, cap);
  KSDF_HIP_TRY(hipGetLastError());
  return KSDF_OK;
}

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
    if (minb < 32) launch_bucket<16>(A, lists + bs[0], nullptr, bs[1] - bs[0], s);
    if (minb < 64) launch_bucket<32>(A, lists + lo32, nullptr, bs[2] - lo32, s);
    launch_bucket<64>(A, lists + lo64, nullptr, bs[3] - lo64, s);
    launch_bucket<128>(A, lists + bs[3], nullptr, bs[4] - bs[3], s);
    A.list = m->fb_list;
    A.list_count = m->fb_count;
    A.emit32 = 1;
    const int grid = m->n_cells < 2048 ? m->n_cells : 2048;
    hipLaunchKernelGGL(fit64_kernel, dim3(grid), dim3(FIT_THREADS), 0, s, A);
    launch_linv(m, s);
    timer_mark(m, KSDF_TIMER_FIT, 1, s);
  }
  KSDF_HIP_TRY(hipGetLastError());
  return KSDF_OK;
}

}  // namespace ksdf
