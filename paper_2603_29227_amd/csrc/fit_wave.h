// One-wave FP32 fit of a cell with m <= MB <= 64 samples (Sec. IV-B.1, eq.
// log_gp_posterior_mean): the same computation as fit32_cell -- float-float
// assembly of A = K + Sigma, FP32 Cholesky, condition estimate, a = A^{-1} 1 refined
// against the float-float A, the fit's adjoint vectors -- organised for one wave and
// no workgroup barriers.  Lane i owns row i: its row of A (float-float) and of the
// factor L stay in registers (the loops over a row are unrolled, so every index is a
// compile-time constant), and the values other lanes need travel through a small
// per-wave LDS area:
//   * the factorisation is right-looking by columns: at column j lane i scales its
//     entry to L_ij, the column goes to LDS, and every lane applies the rank-1 update
//     a_ik -= L_ij L_kj to its row with the column read back by broadcast loads;
//   * L y = b runs on the register rows (y_j leaves lane j by v_readlane), L^T x = y
//     on the packed factor in LDS (row i is contiguous, so lanes k < i read it
//     without bank conflicts);
//   * A x (power iteration, float-float residuals) reads x by broadcast loads.
// Rows past m are the identity, so a cell is the leading block of an MB x MB
// factorisation.  See fit32_cell for the float-float assembly and refinement.
#pragma once

#include <type_traits>

#include "fit_dev.h"

namespace ksdf {
namespace {

// f(integral_constant<int, I>) for I = B .. E-1, each index a compile-time constant
// (so that register arrays indexed by it are never placed in memory)
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// The per-lane slots are sized for the whole wave: every lane writes its own slot
// (lanes past m carry zeros), whatever MB.
template <int MB>
struct WaveFitLds {
  float4 xh[64];                  // cell-local coordinates (hi) and sigma^2 (hi)
  float4 xl[64];                  // their low parts
  float vh[64], vl[64];           // a vector being broadcast (float-float)
  float col[64];                  // the column of the factorisation step
  float L[MB * (MB + 1) / 2];     // packed factor rows, reciprocal diagonal
};

// LDS traffic between the lanes of one wave: order the writes before the reads.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int MB>
struct WaveFit {
  WaveFitLds<MB>& S;
  int lane, m;
  float ah[MB], al[MB];   // row `lane` of A (float-float); identity past m
  float Lr[MB];           // row `lane` of L (entries past the diagonal are scratch)
  float rd;               // 1 / L_ii

  __device__ __forceinline__ WaveFit(WaveFitLds<MB>& s, int m_)
      : S(s), lane(threadIdx.x & 63), m(m_) {}

  // y = L^{-1} b for the lane's entry b (lanes >= m carry 0)
  __device__ __forceinline__ float forward(float b) const {
    float r = b, y = 0.f;
    static_for<0, MB>([&](auto J) {
      constexpr int j = J;
      if (j < m) {   // uniform
        const float yj = readlane(r * rd, j);
        if (lane == j) y = yj;
        r = fmaf(-Lr[j], yj, r);   // meaningful for lanes > j only
      }
    });
    return y;
  }

  // x = L^{-T} y from the packed factor in LDS
  __device__ __forceinline__ float backward(float y) const {
    float r = y, x = 0.f;
    for (int i = m - 1; i >= 0; --i) {
      const float* row = S.L + pk(i, 0);
      const float xi = readlane(r, i) * row[i];
      if (lane == i) x = xi;
      if (lane < i) r = fmaf(-row[lane], xi, r);
    }
    return x;
  }

  __device__ __forceinline__ float solve(float b) const { return backward(forward(b)); }

  // (A x)_lane with the FP32 leading parts
  __device__ __forceinline__ float matvec(float x) const {
    S.vh[lane] = x;
    wave_lds_sync();
    float y = 0.f;
    static_for<0, MB>([&](auto K) { y = fmaf(ah[K], S.vh[K], y); });
    wave_lds_sync();
    return y;
  }

  // rhs - (A x)_lane in float-float, x a float-float vector
  __device__ __forceinline__ ff residual(ff rhs, ff x) const {
    S.vh[lane] = x.hi;
    S.vl[lane] = x.lo;
    wave_lds_sync();
    ff acc = rhs;
    static_for<0, MB>([&](auto K) {
      acc = ff_add(acc, ff_neg(ff_mul(ff{ah[K], al[K]}, ff{S.vh[K], S.vl[K]})));
    });
    wave_lds_sync();
    return acc;
  }

  // x = A^{-1} rhs refined against the float-float A until a correction is below tol
  // of |x| or stops shrinking (the same rule as ff_refined_solve)
  __device__ __forceinline__ ff refined_solve(ff rhs, float tol) const {
    ff x{solve(lane < m ? rhs.hi : 0.f), 0.f};
    float prev = INFINITY;
    for (int it = 0; it < REFINE_MAX; ++it) {
      const ff r = residual(rhs, x);
      const float d = solve(lane < m ? r.hi + r.lo : 0.f);
      x = ff_add(x, ff{d, 0.f});
      const float dn = wave_max(fabsf(d)), xn = wave_max(fabsf(x.hi));
      const bool stop = !(dn > tol * xn) || !(dn < 0.5f * prev);
      prev = dn;
      if (stop) break;
    }
    return x;
  }

  // squared distance of samples `lane` and k, float-float, from the broadcast coordinates
  __device__ __forceinline__ ff dist2(const float xh_[3], const float xl_[3], int k) const {
    const float4 h = S.xh[k], l = S.xl[k];
    const ff dx = ff_add(ff{xh_[0], xl_[0]}, ff{-h.x, -l.x});
    const ff dy = ff_add(ff{xh_[1], xl_[1]}, ff{-h.y, -l.y});
    const ff dz = ff_add(ff{xh_[2], xl_[2]}, ff{-h.z, -l.z});
    return ff_add(ff_add(ff_mul(dx, dx), ff_mul(dy, dy)), ff_mul(dz, dz));
  }
};

// Fit cell c with one wave; returns true when it must be refitted in FP64.
template <int MB>
__device__ __forceinline__ bool fit32_wave(const FitArgs& A, int c, WaveFitLds<MB>& S) {
  const int b = A.offsets[c], m = A.offsets[c + 1] - b;
  WaveFit<MB> W(S, m);
  const int lane = W.lane;
  const bool mine = lane < m;
  // gather: cell-local coordinates, exact as float-float
  float xh[3] = {0.f, 0.f, 0.f}, xl[3] = {0.f, 0.f, 0.f}, svh = 0.f, svl = 0.f;
  if (mine) {
    const long s = A.samples[b + lane];
    if (A.pts_f64) {
      const double* p = static_cast<const double*>(A.pts) + 3 * s;
      for (int d = 0; d < 3; ++d) {
        const double v = p[d] - A.centre64[3 * c + d];
        xh[d] = (float)v;
        xl[d] = (float)(v - (double)xh[d]);
      }
    } else {
      const float* p = static_cast<const float*>(A.pts) + 3 * s;
      for (int d = 0; d < 3; ++d) {
        const ff e = ff_two_sum(p[d], -(float)A.centre64[3 * c + d]);
        xh[d] = e.hi;
        xl[d] = e.lo;
      }
    }
    if (A.svar) {
      if (A.pts_f64) {
        const double v = static_cast<const double*>(A.svar)[s];
        svh = (float)v;
        svl = (float)(v - (double)svh);
      } else {
        svh = static_cast<const float*>(A.svar)[s];
      }
    } else {
      svh = A.noise_ff[0];
      svl = A.noise_ff[1];
    }
  }
  S.xh[lane] = make_float4(xh[0], xh[1], xh[2], svh);
  S.xl[lane] = make_float4(xl[0], xl[1], xl[2], svl);
  wave_lds_sync();
  // A = K + Sigma, row `lane`, float-float
  const bool matern = A.kernel == KSDF_KERNEL_MATERN32;
  const ff inv2l2{A.inv2l2_ff[0], A.inv2l2_ff[1]};
  const ff mc{A.mc_ff[0], A.mc_ff[1]};
  static_for<0, MB>([&](auto K) {
    constexpr int k = K;
    ff v{lane == k ? 1.f : 0.f, 0.f};
    if (mine && k < m) {
      const ff r2 = W.dist2(xh, xl, k);
      if (matern) {
        const ff t = ff_mul(ff_sqrt(r2), mc);
        v = ff_mul(ff_add(ff{1.f, 0.f}, t), ff_exp_neg_fast(t));
      } else {
        v = ff_exp_neg_fast(ff_mul(r2, inv2l2));
      }
      if (k == lane) v = ff_add(v, ff{svh, svl});
    }
    W.ah[k] = v.hi;
    W.al[k] = v.lo;
    W.Lr[k] = v.hi;
  });
  // Cholesky, right-looking by columns
  bool ok = true;
  W.rd = 1.f;
  static_for<0, MB>([&](auto J) {
    constexpr int j = J;
    if (ok && j < m) {   // uniform: a failed pivot stops the factorisation
      const float d = readlane(W.Lr[j], j);
      if (!(d > 0.f)) {
        ok = false;
      } else {
        const float ljj = sqrtf(d), inv = 1.f / ljj;
        const float l = lane > j ? W.Lr[j] * inv : (lane == j ? ljj : 0.f);
        W.Lr[j] = l;
        if (lane == j) W.rd = inv;
        S.col[lane] = l;
        wave_lds_sync();
        static_for<j + 1, MB>([&](auto K) { W.Lr[K] = fmaf(-l, S.col[K], W.Lr[K]); });
        wave_lds_sync();
      }
    }
  });
  // the packed factor (reciprocal diagonal) for the backward solves and the store
  if (ok) {
    static_for<0, MB>([&](auto K) {
      if (K < lane && mine) S.L[pk(lane, K)] = W.Lr[K];
    });
    if (mine) S.L[pk(lane, lane)] = W.rd;
  }
  wave_lds_sync();
  float cond = INFINITY;
  if (ok) {
    // lambda_max by power iteration (ones start), lambda_min by inverse iteration
    // (alternating-sign start): a lower bound of cond_2(A), as cond2_estimate
    float x = mine ? 1.f : 0.f, lmax = 0.f;
    for (int it = 0; it < 4; ++it) {
      const float nx = wave_sum(x * x);
      const float y = W.matvec(x);
      const float xy = wave_sum(x * y), yy = sqrtf(wave_sum(y * y));
      lmax = xy / nx;
      x = y / yy;
    }
    x = mine ? ((lane & 1) ? -1.f : 1.f) : 0.f;
    float inv_lmin = 0.f;
    for (int it = 0; it < 4; ++it) {
      const float nx = sqrtf(wave_sum(x * x));
      const float y = W.solve(x);
      const float ny = sqrtf(wave_sum(y * y));
      inv_lmin = ny / nx;
      x = y / ny;
    }
    cond = lmax * inv_lmin;
  }
  const bool need64 = !ok || !(cond <= (float)A.cond_thr);
  ff a{0.f, 0.f};
  if (!need64) {
    a = W.refined_solve(ff{mine ? 1.f : 0.f, 0.f}, REFINE_TOL);
    if (!mine) a = ff{0.f, 0.f};
    if (A.adjoint) {
      // xi_l = A^{-1} (dA/dl) a with dA_ik/dl = K_ik r_ik^2 / l^3 (RBF) or
      // c^2 r_ik^2 exp(-c r_ik) / l (Matern 3/2); xi_s = A^{-1} a
      S.vh[lane] = a.hi;
      S.vl[lane] = a.lo;
      wave_lds_sync();
      const ff il = matern ? ff{A.inv_l_ff[0], A.inv_l_ff[1]} : ff{A.inv_l3_ff[0], A.inv_l3_ff[1]};
      const ff mc2{A.mc2_ff[0], A.mc2_ff[1]};
      const float il3f = A.inv_l3_ff[0];
      ff g{0.f, 0.f};
      float* Drow = A.D32 ? A.D32 + A.loff[c] + (mine ? pk(lane, 0) : 0) : nullptr;
      static_for<0, MB>([&](auto K) {
        constexpr int k = K;
        if (mine && k < m && k != lane) {
          const ff r2 = W.dist2(xh, xl, k);
          ff dk;
          if (matern) dk = ff_mul(ff_mul(ff_exp_neg_fast(ff_mul(ff_sqrt(r2), mc)), r2), mc2);
          else dk = ff_mul(ff{W.ah[k], W.al[k]}, r2);
          g = ff_add(g, ff_mul(dk, ff{S.vh[k], S.vl[k]}));
          if (Drow && k < lane)
            Drow[k] = matern ? A.mc2_ff[0] * r2.hi * expf(-A.mc_ff[0] * sqrtf(r2.hi)) * A.inv_l_ff[0]
                             : W.ah[k] * r2.hi * il3f;
        }
      });
      if (Drow && mine) Drow[lane] = 0.f;
      wave_lds_sync();
      g = ff_mul(g, il);
      const ff xil = W.refined_solve(mine ? g : ff{0.f, 0.f}, REFINE_TOL_ADJOINT);
      ff xis{0.f, 0.f};
      if (!A.svar) xis = W.refined_solve(a, REFINE_TOL_ADJOINT);
      if (mine) {
        float4 xv;
        xv.x = xil.hi;
        xv.y = A.svar ? 0.f : xis.hi;
        xv.z = xil.lo;
        xv.w = A.svar ? 0.f : xis.lo;
        reinterpret_cast<float4*>(A.xi32)[b + lane] = xv;
      }
    }
  }
  // the per-cell store: (p, a) with low parts, sigma^2, factor rows, box and A+
  if (mine) {
    reinterpret_cast<float4*>(A.ps32)[b + lane] = make_float4(xh[0], xh[1], xh[2], need64 ? 0.f : a.hi);
    reinterpret_cast<float4*>(A.plo32)[b + lane] = make_float4(xl[0], xl[1], xl[2], need64 ? 0.f : a.lo);
    A.sv32[b + lane] = svh;
    float* Lrow = A.L32 + A.loff[c] + pk(lane, 0);
    static_for<0, MB>([&](auto K) {
      if (K < lane) Lrow[K] = need64 ? 0.f : W.Lr[K];
    });
    Lrow[lane] = need64 ? 1.f : W.rd;
  }
  const float apos = wave_sum(mine && !need64 ? fmaxf(a.hi, 0.f) : 0.f);
  float lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = wave_min(mine ? xh[d] : 1e30f);
    hi[d] = wave_max(mine ? xh[d] : -1e30f);
  }
  if (lane == 0) {
    float* box = A.box32 + 8L * c;
    box[0] = lo[0]; box[1] = lo[1]; box[2] = lo[2];
    box[3] = apos;
    box[4] = hi[0]; box[5] = hi[1]; box[6] = hi[2];
    box[7] = 0.f;
    A.cond32[c] = cond;
    A.cstatus[c] = 0;
    if (A.user_status && !need64) A.user_status[c] = 0;
  }
  return need64;
}

}  // namespace
}  // namespace ksdf
