// Device bodies of the per-cell log-GP fit, shared by the fit kernels and the
// persistent fused fit+query kernel.  See fit.hip for the method.
#pragma once

#include "ff.h"
#include "ksdf_internal.h"

namespace ksdf {
namespace {


constexpr int MAXM = KSDF_MAX_M;
constexpr int SLOTS = MAXM / 64;

__device__ __forceinline__ long pk(int i, int k) { return (long)i * (i + 1) / 2 + k; }

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}
template <class T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}

// Vectors of length <= MAXM held across one wave: element k in lane k % 64, slot k / 64.
template <class T>
struct WVec {
  T s[SLOTS];
};

// Element k of v (k the same in every lane) broadcast to every lane by v_readlane.
__device__ __forceinline__ float readlane(float x, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
}
__device__ __forceinline__ double readlane(double x, int l) {
  const long long u = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
template <class T>
__device__ __forceinline__ T wget(const WVec<T>& v, int k) {
  T x = v.s[0];
#pragma unroll
  for (int t = 1; t < SLOTS; ++t)
    if (k / 64 == t) x = v.s[t];
  return readlane(x, k % 64);
}

// Solve L y = b (L packed lower with its true diagonal), wave-cooperative, column
// by column: y_j leaves the residual's lane j by v_readlane, and every lane i > j
// subtracts L_ij y_j from its own entry, so a step costs one broadcast and one FMA
// per slot instead of a cross-lane reduction.
template <class T>
__device__ void wave_forward(const T* Lp, int m, const WVec<T>& b, WVec<T>& y) {
  const int lane = threadIdx.x & 63;
  WVec<T> r = b;
#pragma unroll
  for (int t = 0; t < SLOTS; ++t) y.s[t] = T(0);
  for (int j = 0; j < m; ++j) {
    const T yj = wget(r, j) / Lp[pk(j, j)];
    if (lane == j % 64) y.s[j / 64] = yj;
#pragma unroll
    for (int t = 0; t < SLOTS; ++t) {
      const int i = t * 64 + lane;
      if (i > j && i < m) r.s[t] -= Lp[pk(i, j)] * yj;
    }
  }
}

// Solve L^T x = y, wave-cooperative, last unknown first: x_i leaves lane i by
// v_readlane and every lane k < i subtracts L_ik x_i (row i of L, contiguous).
template <class T>
__device__ void wave_backward(const T* Lp, int m, const WVec<T>& y, WVec<T>& x) {
  const int lane = threadIdx.x & 63;
  WVec<T> r = y;
#pragma unroll
  for (int t = 0; t < SLOTS; ++t) x.s[t] = T(0);
  for (int i = m - 1; i >= 0; --i) {
    const T* row = Lp + pk(i, 0);
    const T xi = wget(r, i) / row[i];
    if (lane == i % 64) x.s[i / 64] = xi;
#pragma unroll
    for (int t = 0; t < SLOTS; ++t) {
      const int k = t * 64 + lane;
      if (k < i) r.s[t] -= row[k] * xi;
    }
  }
}

// y = A x for the packed symmetric A, wave-cooperative, column by column.
template <class T>
__device__ void wave_matvec(const T* Ap, int m, const WVec<T>& x, WVec<T>& y) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < SLOTS; ++t) y.s[t] = T(0);
  for (int j = 0; j < m; ++j) {
    const T xj = wget(x, j);
#pragma unroll
    for (int t = 0; t < SLOTS; ++t) {
      const int i = t * 64 + lane;
      if (i < m) y.s[t] += (i >= j ? Ap[pk(i, j)] : Ap[pk(j, i)]) * xj;
    }
  }
}

// 2-norm condition estimate of SPD A: lambda_max by power iteration with Rayleigh
// quotients on the packed A (entries all positive, so the start vector of ones is
// close to the Perron vector), lambda_min by inverse iteration through the factor
// from an alternating-sign start.  Both converge from below, so the estimate is a
// lower bound of cond_2(A) that tightens with the step count.
template <class T>
__device__ T cond2_estimate(const T* Ap, const T* Lp, int m) {
  const int lane = threadIdx.x & 63;
  WVec<T> x, y, tmp;
#pragma unroll
  for (int t = 0; t < SLOTS; ++t) x.s[t] = (t * 64 + lane < m) ? T(1) : T(0);
  T lmax = T(0);
  for (int it = 0; it < 4; ++it) {
    T nx = T(0);
#pragma unroll
    for (int t = 0; t < SLOTS; ++t) {
      nx += x.s[t] * x.s[t];
      y.s[t] = T(0);   // entries k >= m stay zero
    }
    nx = sqrt(wave_sum(nx));
    wave_matvec(Ap, m, x, y);
    T xy = T(0), yy = T(0);
#pragma unroll
    for (int t = 0; t < SLOTS; ++t) {
      xy += x.s[t] * y.s[t];
      yy += y.s[t] * y.s[t];
    }
    xy = wave_sum(xy);
    yy = sqrt(wave_sum(yy));
    lmax = xy / (nx * nx);
#pragma unroll
    for (int t = 0; t < SLOTS; ++t) x.s[t] = y.s[t] / yy;
  }
  // inverse iteration
#pragma unroll
  for (int t = 0; t < SLOTS; ++t) {
    const int k = t * 64 + lane;
    x.s[t] = (k < m) ? ((k & 1) ? T(-1) : T(1)) : T(0);
  }
  T inv_lmin = T(0);
  for (int it = 0; it < 4; ++it) {
    T nx = T(0);
#pragma unroll
    for (int t = 0; t < SLOTS; ++t) nx += x.s[t] * x.s[t];
    nx = sqrt(wave_sum(nx));
    wave_forward(Lp, m, x, tmp);
    wave_backward(Lp, m, tmp, y);
    T ny = T(0);
#pragma unroll
    for (int t = 0; t < SLOTS; ++t) ny += y.s[t] * y.s[t];
    ny = sqrt(wave_sum(ny));
    inv_lmin = ny / nx;
#pragma unroll
    for (int t = 0; t < SLOTS; ++t) x.s[t] = y.s[t] / ny;
  }
  return lmax * inv_lmin;
}

template <class P>
__device__ __forceinline__ double load_coord(const void* pts, int pts_f64, long s, int d) {
  return pts_f64 ? static_cast<const double*>(pts)[3 * s + d]
                 : (double)static_cast<const float*>(pts)[3 * s + d];
}

struct FitArgs {
  const void* pts;
  int pts_f64;
  const void* svar;         // per-sample variance (same dtype as pts) or null
  const int* offsets;
  const int* samples;
  const long* loff;
  const double* centre64;
  double ell, noise, cond_thr;
  float noise_ff[2];     // sigma^2, 1/(2 l^2) and 1/l^3 as float-float pairs
  float inv2l2_ff[2];
  float inv_l3_ff[2];
  int kernel;            // KSDF_KERNEL_* (Table I)
  float mc_ff[2];        // Matern 3/2 rate c = sqrt(3) / l, float-float
  float mc2_ff[2];       // c^2 and 1 / l, float-float (Matern adjoint)
  float inv_l_ff[2];
  int adjoint;           // also prepare the adjoint vectors xi (and D when non-null)
  float* xi32;           // [nnz+pad,4] (xi_l, xi_s) as float-float: hi_l, hi_s, lo_l, lo_s
  float* D32;            // packed dA/dl or null
  double* xi64;
  double* D64;
  // FP32 store
  float* ps32;
  float* plo32;
  float* sv32;
  float* L32;
  float* box32;
  float* cond32;
  int* fb_list;
  int* fb_count;
  // FP64 store
  double* ps64;
  double* sv64;
  double* L64;
  uint8_t* cstatus;
  uint8_t* user_status;
  // FP64 kernel: cells to process (null = all cells) and whether to emit the FP32 store
  const int* list;
  const int* list_count;
  int n_cells;
  int emit32;
};

// Block-parallel right-looking Cholesky of packed lower Ap (in place); returns
// false (uniformly across the block) on a non-positive pivot.
template <class T>
__device__ bool block_cholesky(T* Ap, int m) {
  const int tid = threadIdx.x;
  for (int j = 0; j < m; ++j) {
    __syncthreads();
    const T d = Ap[pk(j, j)];
    if (!(d > T(0))) return false;
    const T ljj = sqrt(d);
    const T inv = T(1) / ljj;
    __syncthreads();
    for (int i = j + 1 + tid; i < m; i += blockDim.x) Ap[pk(i, j)] *= inv;
    if (tid == 0) Ap[pk(j, j)] = ljj;
    __syncthreads();
    const int r0 = j + 1 + tid / 16, c0 = j + 1 + (tid & 15);
    for (int r = r0; r < m; r += blockDim.x / 16) {
      const T lrj = Ap[pk(r, j)];
      for (int c = c0; c <= r; c += 16) Ap[pk(r, c)] -= lrj * Ap[pk(c, j)];
    }
  }
  __syncthreads();
  return true;
}

// Assemble A = K + Sigma (packed lower) from cell-local coordinates xs.
// Matern 3/2 kernels take k = (1 + c r) exp(-c r) (mc = c); RBF exp(-r^2 inv2l2).
template <class T>
__device__ void assemble(T* Ap, const T* xs, const T* sv, int m, T inv2l2, int kernel, T mc) {
  const int n = m * (m + 1) / 2;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    // invert the packed index: row i with i(i+1)/2 <= e
    int i = (int)((sqrt(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    while ((long)i * (i + 1) / 2 > e) --i;
    while ((long)(i + 1) * (i + 2) / 2 <= e) ++i;
    const int k = e - i * (i + 1) / 2;
    const T dx = xs[3 * i] - xs[3 * k], dy = xs[3 * i + 1] - xs[3 * k + 1], dz = xs[3 * i + 2] - xs[3 * k + 2];
    const T r2 = dx * dx + dy * dy + dz * dz;
    T v;
    if (kernel == KSDF_KERNEL_MATERN32) {
      const T t = mc * sqrt(r2);
      v = (T(1) + t) * exp(-t);
    } else {
      v = exp(-r2 * inv2l2);
    }
    if (i == k) v += sv[i];
    Ap[e] = v;
  }
}

// Per-cell epilogue shared by both precisions: weights, bounding box, A+ and the
// packed factor with reciprocal diagonal, written in the output precision O.
__device__ __forceinline__ float lo_part(float) { return 0.f; }
__device__ __forceinline__ float lo_part(double v) { return (float)(v - (double)(float)v); }

// plo (optional): float-float low parts of (p, a) for the FP32 store; xlo / alo give
// them directly (FP32 fit) or, when null, they are split from the FP64 values.
template <class T, class O>
__device__ void write_cell(const T* Lp, const T* xs, const T* sv, const WVec<T>& a, int m, bool ok,
                           O* ps, O* svo, O* Lo, float* box, float* plo = nullptr,
                           const float* xlo = nullptr, const float* alo = nullptr) {
  const int lane = threadIdx.x & 63;
  if (threadIdx.x < 64) {
    T apos = T(0);
    T lo[3] = {T(1e30), T(1e30), T(1e30)}, hi[3] = {T(-1e30), T(-1e30), T(-1e30)};
#pragma unroll
    for (int t = 0; t < SLOTS; ++t) {
      const int i = t * 64 + lane;
      if (i < m) {
        const T ai = ok ? a.s[t] : T(0);
        ps[4 * i + 0] = (O)xs[3 * i];
        ps[4 * i + 1] = (O)xs[3 * i + 1];
        ps[4 * i + 2] = (O)xs[3 * i + 2];
        ps[4 * i + 3] = (O)ai;
        svo[i] = (O)sv[i];
        if (plo) {
          plo[4 * i + 0] = xlo ? xlo[3 * i] : lo_part(xs[3 * i]);
          plo[4 * i + 1] = xlo ? xlo[3 * i + 1] : lo_part(xs[3 * i + 1]);
          plo[4 * i + 2] = xlo ? xlo[3 * i + 2] : lo_part(xs[3 * i + 2]);
          plo[4 * i + 3] = ok ? (alo ? alo[i] : lo_part(ai)) : 0.f;
        }
        apos += ai > T(0) ? ai : T(0);
        for (int d = 0; d < 3; ++d) {
          lo[d] = min(lo[d], xs[3 * i + d]);
          hi[d] = max(hi[d], xs[3 * i + d]);
        }
      }
    }
    apos = wave_sum(apos);
    for (int d = 0; d < 3; ++d) {
      lo[d] = wave_min(lo[d]);
      hi[d] = wave_max(hi[d]);
    }
    if (lane == 0 && box) {
      box[0] = (float)lo[0]; box[1] = (float)lo[1]; box[2] = (float)lo[2];
      box[3] = (float)apos;
      box[4] = (float)hi[0]; box[5] = (float)hi[1]; box[6] = (float)hi[2];
      box[7] = 0.f;
    }
  }
  const int n = m * (m + 1) / 2;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    int i = (int)((sqrt(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    while ((long)i * (i + 1) / 2 > e) --i;
    while ((long)(i + 1) * (i + 2) / 2 <= e) ++i;
    const int k = e - i * (i + 1) / 2;
    const T v = ok ? Lp[e] : T(1);
    Lo[e] = (O)((i == k) ? T(1) / v : (ok ? v : T(0)));
  }
}

// Block-cooperative float-float row sums: row i of the m rows is shared by G
// consecutive threads (G = blockDim / (rows rounded up to a power of two), at most
// 16, a divisor of 64), each summing the terms k = part, part + G, ...; the G
// partials are combined by lane shuffles.  term(i, k) returns the ff term; every
// thread of the block must call it.  The row's sum goes to out(i, sum) on part 0.
template <class Term, class Out>
__device__ __forceinline__ void ff_row_sums(int m, Term term, Out out) {
  int mp = 1;
  while (mp < m) mp <<= 1;
  int G = (int)blockDim.x / mp;
  G = G < 1 ? 1 : (G > 16 ? 16 : G);
  const int part = threadIdx.x % G;
  const int rows_per_pass = blockDim.x / G;
  for (int base = 0; base < m; base += rows_per_pass) {
    const int i = base + (int)threadIdx.x / G;
    ff acc{0.f, 0.f};
    if (i < m)
      for (int k = part; k < m; k += G) acc = ff_add(acc, term(i, k));
    for (int o = 1; o < G; o <<= 1) {
      const ff other{__shfl_xor(acc.hi, o, 64), __shfl_xor(acc.lo, o, 64)};
      acc = ff_add(acc, other);
    }
    if (i < m && part == 0) out(i, acc);
  }
}

// Solve A x = rhs for the cell (block-cooperative): an FP32 solve with the factor,
// then refinement steps whose residuals rhs - A x are evaluated in float-float from
// (Ahi, Alo), until a correction is below tol (REFINE_TOL) of |x| or no longer shrinks
// (the float-float residual's own accuracy is reached), at most REFINE_MAX steps;
// each step shrinks the error by about cond(A) * 2^-24.  rhs (rh, rl) and
// x (xh, xl) are float-float arrays in LDS; res is scratch.  Ends with a barrier.
constexpr int REFINE_MAX = 10;
constexpr float REFINE_TOL = 1e-10f;
// The fit's adjoint vectors enter only the hyperparameter gradient, whose FP32 bound
// is 1e-3 relative: 1e-7 of |x| is ample there and saves refinement steps.
constexpr float REFINE_TOL_ADJOINT = 1e-7f;
__device__ void ff_refined_solve(const float* Ahi, const float* Alo, const float* Lf, int m,
                                 const float* rh, const float* rl, float* xh, float* xl,
                                 float* res, float tol = REFINE_TOL) {
  const int lane = threadIdx.x & 63;
  __shared__ int converged;
  float prev = INFINITY;   // last correction (wave 0)
  __syncthreads();
  if (threadIdx.x < 64) {
    WVec<float> rv, y, x0;
#pragma unroll
    for (int t = 0; t < SLOTS; ++t) {
      const int i = t * 64 + lane;
      rv.s[t] = i < m ? rh[i] : 0.f;
    }
    wave_forward<float>(Lf, m, rv, y);
    wave_backward<float>(Lf, m, y, x0);
#pragma unroll
    for (int t = 0; t < SLOTS; ++t) {
      const int i = t * 64 + lane;
      if (i < m) {
        xh[i] = x0.s[t];
        xl[i] = 0.f;
      }
    }
  }
  __syncthreads();
  for (int it = 0; it < REFINE_MAX; ++it) {
    ff_row_sums(
        m,
        [&](int i, int k) {
          const long e = k <= i ? pk(i, k) : pk(k, i);
          return ff_mul(ff{Ahi[e], Alo[e]}, ff{xh[k], xl[k]});
        },
        [&](int i, ff acc) {
          const ff r = ff_add(ff{rh[i], rl[i]}, ff_neg(acc));
          res[i] = r.hi + r.lo;
        });
    __syncthreads();
    if (threadIdx.x < 64) {
      WVec<float> rv, y, dlt;
#pragma unroll
      for (int t = 0; t < SLOTS; ++t) {
        const int i = t * 64 + lane;
        rv.s[t] = i < m ? res[i] : 0.f;
      }
      wave_forward<float>(Lf, m, rv, y);
      wave_backward<float>(Lf, m, y, dlt);
      float dn = 0.f, xn = 0.f;
#pragma unroll
      for (int t = 0; t < SLOTS; ++t) {
        const int i = t * 64 + lane;
        if (i < m) {
          const ff x2 = ff_add(ff{xh[i], xl[i]}, ff{dlt.s[t], 0.f});
          xh[i] = x2.hi;
          xl[i] = x2.lo;
          dn = fmaxf(dn, fabsf(dlt.s[t]));
          xn = fmaxf(xn, fabsf(x2.hi));
        }
      }
      dn = wave_max(dn);
      xn = wave_max(xn);
      if (threadIdx.x == 0) converged = !(dn > tol * xn) || !(dn < 0.5f * prev);
      prev = dn;
    }
    __syncthreads();
    if (converged) break;
  }
}

// FP32 fit with mixed-precision iterative refinement.  A is assembled once in
// float-float (about 44 bits: exact cell-local differences, a float-float exp),
// its leading float part is factored in FP32, and a = A^{-1} 1 is refined with
// residuals r = 1 - A a evaluated in float-float and corrections solved with the
// FP32 factor.  Each step shrinks the error by about cond(A) * 2^-24; the steps
// continue until a reaches the accuracy of its float-float residual, and a is kept
// as a float-float pair.  MB is the bucket's largest m and sizes the LDS arrays.
template <int MB>
__host__ __device__ constexpr int fit32_smem_floats() {
  return 3 * (MB * (MB + 1) / 2) + 6 * MB + 10 * MB + 4;
}

// Fit one cell with the whole block; smem holds fit32_smem_floats<MB>() floats.
// Returns true when the cell must be refitted in FP64 (failed pivot or condition
// estimate above the threshold); its FP32 store then holds zero weights.
template <int MB>
__device__ bool fit32_cell(const FitArgs& A, int c, float* smem) {
  constexpr int NP = MB * (MB + 1) / 2;
  float* Ahi = smem;
  float* Alo = Ahi + NP;
  float* Lf = Alo + NP;
  float* xh = Lf + NP;
  float* xl = xh + 3 * MB;
  float* sv = xl + 3 * MB;
  float* svl = sv + MB;
  float* ah = svl + MB;
  float* al = ah + MB;
  float* res = al + MB;
  float* rh = res + MB;
  float* rl = rh + MB;
  float* xih = rl + MB;
  float* xil = xih + MB;
  float& cond_sh = xil[MB];
  __syncthreads();   // the previous task of this block may still read smem
  const int b = A.offsets[c], m = A.offsets[c + 1] - b;
  const float cx = (float)A.centre64[3 * c], cy = (float)A.centre64[3 * c + 1], cz = (float)A.centre64[3 * c + 2];
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const long s = A.samples[b + i];
    if (A.pts_f64) {
      const double* p = static_cast<const double*>(A.pts) + 3 * s;
      for (int d = 0; d < 3; ++d) {
        const double v = p[d] - A.centre64[3 * c + d];
        xh[3 * i + d] = (float)v;
        xl[3 * i + d] = (float)(v - (double)(float)v);
      }
    } else {
      const float* p = static_cast<const float*>(A.pts) + 3 * s;
      // cell-local coordinates, exact as float-float
      const ff ex = ff_two_sum(p[0], -cx), ey = ff_two_sum(p[1], -cy), ez = ff_two_sum(p[2], -cz);
      xh[3 * i] = ex.hi; xl[3 * i] = ex.lo;
      xh[3 * i + 1] = ey.hi; xl[3 * i + 1] = ey.lo;
      xh[3 * i + 2] = ez.hi; xl[3 * i + 2] = ez.lo;
    }
    if (A.svar) {
      sv[i] = A.pts_f64 ? (float)static_cast<const double*>(A.svar)[s] : static_cast<const float*>(A.svar)[s];
      svl[i] = A.pts_f64 ? (float)(static_cast<const double*>(A.svar)[s] - (double)sv[i]) : 0.f;
    } else {
      sv[i] = A.noise_ff[0];
      svl[i] = A.noise_ff[1];
    }
  }
  __syncthreads();
  // A = K + Sigma in float-float
  const ff inv2l2{A.inv2l2_ff[0], A.inv2l2_ff[1]};
  const ff mc{A.mc_ff[0], A.mc_ff[1]};
  for (int e = threadIdx.x; e < m * (m + 1) / 2; e += blockDim.x) {
    int i = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    while (i * (i + 1) / 2 > e) --i;
    while ((i + 1) * (i + 2) / 2 <= e) ++i;
    const int k = e - i * (i + 1) / 2;
    ff r2{0.f, 0.f};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const ff dd = ff_add(ff{xh[3 * i + d], xl[3 * i + d]}, ff{-xh[3 * k + d], -xl[3 * k + d]});
      r2 = ff_add(r2, ff_mul(dd, dd));
    }
    ff v;
    if (A.kernel == KSDF_KERNEL_MATERN32) {
      // (1 + c r) exp(-c r), exactly 1 at r = 0
      const ff t = ff_mul(ff_sqrt(r2), mc);
      v = ff_mul(ff_add(ff{1.f, 0.f}, t), ff_exp_neg_tab(t));
    } else {
      v = ff_exp_neg_tab(ff_mul(r2, inv2l2));
    }
    if (i == k) v = ff_add(v, ff{sv[i], svl[i]});
    Ahi[e] = v.hi;
    Alo[e] = v.lo;
    Lf[e] = v.hi;
  }
  __syncthreads();
  const bool ok = block_cholesky<float>(Lf, m);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  if (threadIdx.x < 64) {
    float cond = INFINITY;
    if (ok) {
      cond = cond2_estimate<float>(Ahi, Lf, m);
    }
    if (threadIdx.x == 0) cond_sh = cond;
  }
  __syncthreads();
  const float cond = cond_sh;
  const bool need64 = !ok || !(cond <= (float)A.cond_thr);
  if (!need64) {
    // a = A^{-1} 1
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
      rh[i] = 1.f;
      rl[i] = 0.f;
    }
    ff_refined_solve(Ahi, Alo, Lf, m, rh, rl, ah, al, res);
    if (A.adjoint) {
      // adjoint vectors of the fit: xi_l = A^{-1} (dA/dl) a with dA_ij/dl = K_ij r_ij^2 / l^3
      // (RBF) or c^2 r_ij^2 exp(-c r_ij) / l (Matern 3/2), and xi_s = A^{-1} a
      // (dA/dsigma^2 = I for the uniform noise variance)
      const bool matern = A.kernel == KSDF_KERNEL_MATERN32;
      const ff il3 = matern ? ff{A.inv_l_ff[0], A.inv_l_ff[1]} : ff{A.inv_l3_ff[0], A.inv_l3_ff[1]};
      const ff mcf{A.mc_ff[0], A.mc_ff[1]}, mc2f{A.mc2_ff[0], A.mc2_ff[1]};
      ff_row_sums(
          m,
          [&](int i, int k) {
            if (k == i) return ff{0.f, 0.f};
            const long e = k <= i ? pk(i, k) : pk(k, i);
            ff r2{0.f, 0.f};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const ff dd = ff_add(ff{xh[3 * i + d], xl[3 * i + d]}, ff{-xh[3 * k + d], -xl[3 * k + d]});
              r2 = ff_add(r2, ff_mul(dd, dd));
            }
            if (matern) {
              const ff ecr = ff_exp_neg_tab(ff_mul(ff_sqrt(r2), mcf));
              return ff_mul(ff_mul(ff_mul(ecr, r2), mc2f), ff{ah[k], al[k]});
            }
            return ff_mul(ff_mul(ff{Ahi[e], Alo[e]}, r2), ff{ah[k], al[k]});
          },
          [&](int i, ff acc) {
            const ff g = ff_mul(acc, il3);
            rh[i] = g.hi;
            rl[i] = g.lo;
          });
      ff_refined_solve(Ahi, Alo, Lf, m, rh, rl, xih, xil, res, REFINE_TOL_ADJOINT);
      for (int i = threadIdx.x; i < m; i += blockDim.x) {
        A.xi32[4L * (b + i)] = xih[i];
        A.xi32[4L * (b + i) + 2] = xil[i];
      }
      if (!A.svar) {
        __syncthreads();
        for (int i = threadIdx.x; i < m; i += blockDim.x) {
          rh[i] = ah[i];
          rl[i] = al[i];
        }
        ff_refined_solve(Ahi, Alo, Lf, m, rh, rl, xih, xil, res, REFINE_TOL_ADJOINT);
      }
      for (int i = threadIdx.x; i < m; i += blockDim.x) {
        A.xi32[4L * (b + i) + 1] = A.svar ? 0.f : xih[i];
        A.xi32[4L * (b + i) + 3] = A.svar ? 0.f : xil[i];
      }
      if (A.D32) {
        const float il3f = A.inv_l3_ff[0];
        for (int e = threadIdx.x; e < m * (m + 1) / 2; e += blockDim.x) {
          int i = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
          while (i * (i + 1) / 2 > e) --i;
          while ((i + 1) * (i + 2) / 2 <= e) ++i;
          const int k = e - i * (i + 1) / 2;
          float r2 = 0.f;
          for (int d = 0; d < 3; ++d) {
            const float dd = (xh[3 * i + d] - xh[3 * k + d]) + (xl[3 * i + d] - xl[3 * k + d]);
            r2 += dd * dd;
          }
          if (matern) {
            const float mcv = A.mc_ff[0], r = sqrtf(r2);
            A.D32[A.loff[c] + e] = (i == k) ? 0.f : A.mc2_ff[0] * r2 * expf(-mcv * r) * A.inv_l_ff[0];
          } else {
            A.D32[A.loff[c] + e] = (i == k) ? 0.f : Ahi[e] * r2 * il3f;
          }
        }
      }
    }
  }
  WVec<float> a;
#pragma unroll
  for (int t = 0; t < SLOTS; ++t) {
    const int i = t * 64 + lane;
    a.s[t] = (i < m) ? ah[i] : 0.f;
  }
  write_cell<float, float>(Lf, xh, sv, a, m, ok && !need64, A.ps32 + 4L * b, A.sv32 + b,
                           A.L32 + A.loff[c], A.box32 + 8L * c, A.plo32 + 4L * b, xl, al);
  if (threadIdx.x == 0) {
    A.cond32[c] = cond;
    A.cstatus[c] = 0;
    if (A.user_status && !need64) A.user_status[c] = 0;
  }
  return need64;
}

constexpr int FIT64_SMEM_DOUBLES = 6 * MAXM;

// Fit one cell in FP64 with the whole block (factor in place in global memory);
// smem holds FIT64_SMEM_DOUBLES doubles.  emit32 writes the FP32 store.
__device__ void fit64_cell(const FitArgs& A, int c, double* smem) {
  double* xs = smem;
  double* sv = xs + 3 * MAXM;
  double* a_s = sv + MAXM;
  double* g_s = a_s + MAXM;
  {
    const int b = A.offsets[c], m = A.offsets[c + 1] - b;
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
      const long s = A.samples[b + i];
      for (int d = 0; d < 3; ++d)
        xs[3 * i + d] = load_coord<double>(A.pts, A.pts_f64, s, d) - A.centre64[3 * c + d];
      sv[i] = A.svar ? (A.pts_f64 ? static_cast<const double*>(A.svar)[s]
                                  : (double)static_cast<const float*>(A.svar)[s])
                     : A.noise;
    }
    __syncthreads();
    double* Ap = A.L64 + A.loff[c];   // the factor is computed in place in global memory
    assemble<double>(Ap, xs, sv, m, 1.0 / (2.0 * A.ell * A.ell), A.kernel, std::sqrt(3.0) / A.ell);
    __threadfence_block();
    const bool ok = block_cholesky<double>(Ap, m);
    __threadfence_block();
    __syncthreads();
    WVec<double> a;
    if (threadIdx.x < 64 && ok) {
      WVec<double> ones, y;
#pragma unroll
      for (int s2 = 0; s2 < SLOTS; ++s2) ones.s[s2] = 1.0;
      wave_forward<double>(Ap, m, ones, y);
      wave_backward<double>(Ap, m, y, a);
    }
    __syncthreads();
    if (A.adjoint && ok) {
      // adjoint vectors of the fit in FP64: xi_l = A^{-1} (dA/dl) a, xi_s = A^{-1} a
      const int lane = threadIdx.x & 63;
      if (threadIdx.x < 64) {
#pragma unroll
        for (int t2 = 0; t2 < SLOTS; ++t2) {
          const int i = t2 * 64 + lane;
          if (i < m) a_s[i] = a.s[t2];
        }
      }
      __syncthreads();
      const double inv2l2 = 1.0 / (2.0 * A.ell * A.ell), il3 = 1.0 / (A.ell * A.ell * A.ell);
      const bool matern = A.kernel == KSDF_KERNEL_MATERN32;
      const double mcd = std::sqrt(3.0) / A.ell;
      // dA_ij/dl without the 1/l^3 (RBF) or 1/l (Matern 3/2) factor
      auto dkl = [&](double r2) {
        return matern ? mcd * mcd * r2 * exp(-mcd * sqrt(r2)) : exp(-r2 * inv2l2) * r2;
      };
      const double lfac = matern ? 1.0 / A.ell : il3;
      for (int i = threadIdx.x; i < m; i += blockDim.x) {
        double acc = 0.0;
        for (int k = 0; k < m; ++k) {
          if (k == i) continue;
          const double dx = xs[3 * i] - xs[3 * k], dy = xs[3 * i + 1] - xs[3 * k + 1],
                       dz = xs[3 * i + 2] - xs[3 * k + 2];
          const double r2 = dx * dx + dy * dy + dz * dz;
          acc += dkl(r2) * a_s[k];
        }
        g_s[i] = acc * lfac;
      }
      __syncthreads();
      if (threadIdx.x < 64) {
        WVec<double> gv, av, y, xl_, xs_;
#pragma unroll
        for (int t2 = 0; t2 < SLOTS; ++t2) {
          const int i = t2 * 64 + lane;
          gv.s[t2] = i < m ? g_s[i] : 0.0;
          av.s[t2] = i < m ? a_s[i] : 0.0;
        }
        wave_forward<double>(Ap, m, gv, y);
        wave_backward<double>(Ap, m, y, xl_);
        wave_forward<double>(Ap, m, av, y);
        wave_backward<double>(Ap, m, y, xs_);
#pragma unroll
        for (int t2 = 0; t2 < SLOTS; ++t2) {
          const int i = t2 * 64 + lane;
          if (i < m) {
            const double xsv = A.svar ? 0.0 : xs_.s[t2];
            if (A.emit32) {
              const float hl = (float)xl_.s[t2], hs = (float)xsv;
              A.xi32[4L * (b + i)] = hl;
              A.xi32[4L * (b + i) + 1] = hs;
              A.xi32[4L * (b + i) + 2] = (float)(xl_.s[t2] - (double)hl);
              A.xi32[4L * (b + i) + 3] = (float)(xsv - (double)hs);
            } else {
              A.xi64[2L * (b + i)] = xl_.s[t2];
              A.xi64[2L * (b + i) + 1] = xsv;
            }
          }
        }
      }
      if (A.D32 || A.D64) {
        for (int e = threadIdx.x; e < m * (m + 1) / 2; e += blockDim.x) {
          int i = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
          while (i * (i + 1) / 2 > e) --i;
          while ((i + 1) * (i + 2) / 2 <= e) ++i;
          const int k = e - i * (i + 1) / 2;
          const double dx = xs[3 * i] - xs[3 * k], dy = xs[3 * i + 1] - xs[3 * k + 1],
                       dz = xs[3 * i + 2] - xs[3 * k + 2];
          const double r2 = dx * dx + dy * dy + dz * dz;
          const double dv = (i == k) ? 0.0 : dkl(r2) * lfac;
          if (A.emit32) A.D32[A.loff[c] + e] = (float)dv;
          else A.D64[A.loff[c] + e] = dv;
        }
      }
      __syncthreads();
    }
    if (A.emit32) {
      write_cell<double, float>(Ap, xs, sv, a, m, ok, A.ps32 + 4L * b, A.sv32 + b,
                                A.L32 + A.loff[c], A.box32 + 8L * c, A.plo32 + 4L * b);
    } else {
      write_cell<double, double>(Ap, xs, sv, a, m, ok, A.ps64 + 4L * b, A.sv64 + b, Ap,
                                 A.box32 ? A.box32 + 8L * c : nullptr);
    }
    if (threadIdx.x == 0) {
      const uint8_t st = (A.emit32 ? KSDF_C_FP64 : 0) | (ok ? 0 : KSDF_C_FAILED);
      A.cstatus[c] = st;
      if (A.user_status) A.user_status[c] = st;
    }
  }
}


// Arguments of a fit of model m (the FP64 refit list fields are set by the launch).
inline FitArgs make_fit_args(ksdf_model* m, const void* pts, int dtype, const void* svar,
                             uint8_t* user_status) {
  FitArgs A{};
  A.pts = pts;
  A.pts_f64 = dtype == KSDF_DTYPE_F64;
  A.svar = svar;
  A.offsets = m->offsets;
  A.samples = m->samples;
  A.loff = m->loff;
  A.centre64 = m->centre64;
  A.ell = m->ell;
  A.kernel = m->kernel;
  A.noise = m->noise_var;
  A.cond_thr = m->cond_thr;
  A.user_status = user_status;
  A.ps32 = m->ps32; A.plo32 = m->plo32; A.sv32 = m->sv32; A.L32 = m->L32; A.box32 = m->box32; A.cond32 = m->cond32;
  A.fb_list = m->fb_list; A.fb_count = m->fb_count;
  A.ps64 = m->ps64; A.sv64 = m->sv64; A.L64 = m->L64;
  A.cstatus = m->cstatus;
  A.n_cells = m->n_cells;
  A.adjoint = m->adjoint ? 1 : 0;
  A.xi32 = m->xi32;
  A.xi64 = m->xi64;
  A.D32 = m->adjoint_varf ? m->D32 : nullptr;
  A.D64 = m->adjoint_varf ? m->D64 : nullptr;
  {
    const double il3 = 1.0 / (m->ell * m->ell * m->ell);
    A.inv_l3_ff[0] = (float)il3;
    A.inv_l3_ff[1] = (float)(il3 - (double)(float)il3);
    const double inv = 1.0 / (2.0 * m->ell * m->ell);
    A.inv2l2_ff[0] = (float)inv;
    A.inv2l2_ff[1] = (float)(inv - (double)(float)inv);
    const double mc = std::sqrt(3.0) / m->ell;
    A.mc_ff[0] = (float)mc;
    A.mc_ff[1] = (float)(mc - (double)(float)mc);
    const double mc2 = 3.0 / (m->ell * m->ell), il = 1.0 / m->ell;
    A.mc2_ff[0] = (float)mc2;
    A.mc2_ff[1] = (float)(mc2 - (double)(float)mc2);
    A.inv_l_ff[0] = (float)il;
    A.inv_l_ff[1] = (float)(il - (double)(float)il);
    A.noise_ff[0] = (float)m->noise_var;
    A.noise_ff[1] = (float)(m->noise_var - (double)(float)m->noise_var);
  }
  return A;
}

}  // namespace
}  // namespace ksdf
