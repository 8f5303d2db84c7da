// One-wave FP32 fit of a cell with m <= MB <= 64 samples (Sec. IV-B.1, eq.
// log_gp_posterior_mean): float-float assembly of A = K + Sigma, FP32 Cholesky,
// condition estimate, a = A^{-1} 1 refined against the float-float A, and the fit's
// adjoint vectors, organised for one wave and no workgroup barriers.  Lane i owns
// row i: its row of A (float-float) and of the factor L stay in registers (the loops
// over a row are unrolled, so every index is a compile-time constant), and the
// values other lanes need travel through a small per-wave LDS area:
//   * the factorisation is right-looking by columns: at column j lane i scales its
//     entry to L_ij, the column goes to LDS, and every lane applies the rank-1 update
//     a_ik -= L_ij L_kj to its row with the column read back four entries at a time;
//   * the solves run on the packed factor in LDS: L y = b with y_j leaving lane j by
//     v_readlane and each lane reading its own row, L^T x = y with lanes k < i reading
//     row i (contiguous); both without bank conflicts, and with the factor out of the
//     registers, which keeps two waves per SIMD at m = 64;
//   * A x (power iteration) and the residuals b - A x read x four entries at a time.
// The residuals are compensated dot products (Dot2) of the float-float rows with the
// float-float iterate, the kernel entries come from lean float-float helpers (exact
// coordinate differences, TwoProduct squares, a table-driven exp), and the kernel
// function is a template parameter, so the unrolled loops carry no run-time branches
// beyond the uniform "column inside the cell" tests.  Rows past m are the identity, so
// a cell is the leading block of an MB x MB factorisation.
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
// (lanes past m carry zeros), whatever MB.  The packed factor has room for the
// unmasked row reads of the L^T solve (row i, entries 0..63).
template <int MB>
constexpr int wave_lds_l_floats() {
  constexpr int np = MB * (MB + 1) / 2, reach = (MB - 1) * MB / 2 + 64;
  return ((np > reach ? np : reach) + 3) & ~3;
}

template <int MB>
struct WaveFitLds {
  float4 xh[64];                           // cell-local coordinates (hi) and sigma^2 (hi)
  float4 xl[64];                           // their low parts
  alignas(16) float vh[64];                // vectors being broadcast (float-float)
  alignas(16) float vl[64];
  alignas(16) float wh[64];
  alignas(16) float wl[64];
  alignas(16) float col[64];               // the column of the factorisation step
  alignas(16) float L[wave_lds_l_floats<MB>()];   // packed factor rows, reciprocal diagonal
};

// LDS traffic between the lanes of one wave: order the writes before the reads.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// whether packed index e (row-major lower triangle) is a diagonal entry
__device__ __forceinline__ bool packed_diag(int e) {
  int i = (int)((sqrtf(8.f * (float)e + 1.f) - 1.f) * 0.5f);
  if ((i + 1) * (i + 2) / 2 <= e) ++i;
  if (i * (i + 1) / 2 > e) --i;
  return e == i * (i + 3) / 2;
}

template <int MB, bool MATERN>
struct WaveFit {
  WaveFitLds<MB>& S;
  int lane, m;
  float ah[MB], al[MB];   // row `lane` of A (float-float); identity past m
  float Lr[MB];           // row `lane` of L during the factorisation (entries past the
                          // diagonal are scratch); the solves read the packed copy in LDS
  float rd;               // 1 / L_ii

  __device__ __forceinline__ WaveFit(WaveFitLds<MB>& s, int m_)
      : S(s), lane(threadIdx.x & 63), m(m_) {}

  // squared distance of samples `lane` and k, float-float, from the broadcast coordinates
  __device__ __forceinline__ ff dist2(const float xh_[3], const float xl_[3], int k) const {
    const float4 h = S.xh[k], l = S.xl[k];
    return ff_norm2_lean(ff_sub_lean(xh_[0], xl_[0], h.x, l.x), ff_sub_lean(xh_[1], xl_[1], h.y, l.y),
                         ff_sub_lean(xh_[2], xl_[2], h.z, l.z));
  }

  // y = L^{-1} b for the lane's entry b (lanes >= m carry 0), the lane's row of L read
  // from the packed factor in LDS (the rows' starts i(i+1)/2 fall in 32 different
  // banks for 32 consecutive i, so the reads are free of bank conflicts; entries past
  // the diagonal belong to the next row and only reach lanes whose result is taken)
  __device__ __forceinline__ float forward(float b) const {
    const float* row = S.L + (lane < MB ? lane * (lane + 1) / 2 : 0);   // lanes past MB: unused
    float r = b, y = 0.f;
    static_for<0, MB>([&](auto J) {
      constexpr int j = J;
      if (j < m) {   // uniform
        const float yj = readlane(r * rd, j);
        if (lane == j) y = yj;
        r = fmaf(-row[j], yj, r);   // meaningful for lanes > j only
      }
    });
    return y;
  }

  // two right-hand sides at once
  __device__ __forceinline__ void forward2(float b0, float b1, float& y0, float& y1) const {
    const float* row = S.L + (lane < MB ? lane * (lane + 1) / 2 : 0);   // lanes past MB: unused
    float r0 = b0, r1 = b1;
    y0 = 0.f;
    y1 = 0.f;
    static_for<0, MB>([&](auto J) {
      constexpr int j = J;
      if (j < m) {
        const float u0 = readlane(r0 * rd, j), u1 = readlane(r1 * rd, j);
        if (lane == j) {
          y0 = u0;
          y1 = u1;
        }
        const float l = row[j];
        r0 = fmaf(-l, u0, r0);
        r1 = fmaf(-l, u1, r1);
      }
    });
  }

  // x = L^-T y from the packed factor in LDS: lane k < i subtracts L_ik x_i; the other
  // lanes' updates touch entries they no longer use (the reads stay inside L)
  __device__ __forceinline__ float backward(float y) const {
    float r = y, x = 0.f;
    static_for<0, MB>([&](auto I) {
      constexpr int i = MB - 1 - I;
      if (i < m) {
        const float xi = readlane(r * rd, i);
        if (lane == i) x = xi;
        r = fmaf(-S.L[i * (i + 1) / 2 + lane], xi, r);
      }
    });
    return x;
  }

  __device__ __forceinline__ void backward2(float y0, float y1, float& x0, float& x1) const {
    float r0 = y0, r1 = y1;
    x0 = 0.f;
    x1 = 0.f;
    static_for<0, MB>([&](auto I) {
      constexpr int i = MB - 1 - I;
      if (i < m) {
        const float u0 = readlane(r0 * rd, i), u1 = readlane(r1 * rd, i);
        if (lane == i) {
          x0 = u0;
          x1 = u1;
        }
        const float l = S.L[i * (i + 1) / 2 + lane];
        r0 = fmaf(-l, u0, r0);
        r1 = fmaf(-l, u1, r1);
      }
    });
  }

  __device__ __forceinline__ float solve(float b) const { return backward(forward(b)); }

  // (A x)_lane with the FP32 leading parts
  __device__ __forceinline__ float matvec(float x) const {
    S.vh[lane] = x;
    wave_lds_sync();
    float y = 0.f;
    static_for<0, MB / 4>([&](auto G) {
      constexpr int g = G;
      const float4 v = reinterpret_cast<const float4*>(S.vh)[g];
      y = fmaf(ah[4 * g], v.x, y);
      y = fmaf(ah[4 * g + 1], v.y, y);
      y = fmaf(ah[4 * g + 2], v.z, y);
      y = fmaf(ah[4 * g + 3], v.w, y);
    });
    wave_lds_sync();
    return y;
  }

  // rhs - (A x)_lane for the float-float x in (vh, vl), a compensated dot product
  __device__ __forceinline__ ff residual(ff rhs, const float* vh, const float* vl) const {
    float s = rhs.hi, c = rhs.lo;
    static_for<0, MB / 4>([&](auto G) {
      constexpr int g = G;
      const float4 h = reinterpret_cast<const float4*>(vh)[g];
      const float4 l = reinterpret_cast<const float4*>(vl)[g];
      dot2_sub(s, c, ah[4 * g], al[4 * g], h.x, l.x);
      dot2_sub(s, c, ah[4 * g + 1], al[4 * g + 1], h.y, l.y);
      dot2_sub(s, c, ah[4 * g + 2], al[4 * g + 2], h.z, l.z);
      dot2_sub(s, c, ah[4 * g + 3], al[4 * g + 3], h.w, l.w);
    });
    return ff_two_sum(s, c);
  }

  // x = A^{-1} rhs refined against the float-float A: FP32 corrections solved with the
  // factor from float-float residuals, until a correction is below tol of |x| or
  // stops shrinking (each step shrinks the error by about cond(A) 2^-24)
  __device__ __forceinline__ ff refined_solve(ff rhs, float tol) const {
    const bool mine = lane < m;
    ff x{solve(mine ? rhs.hi : 0.f), 0.f};
    float prev = INFINITY;
    for (int it = 0; it < REFINE_MAX; ++it) {
      S.vh[lane] = x.hi;
      S.vl[lane] = x.lo;
      wave_lds_sync();
      const ff r = residual(rhs, S.vh, S.vl);
      wave_lds_sync();
      const float d = solve(mine ? r.hi + r.lo : 0.f);
      x = ff_add(x, ff{d, 0.f});
      const float dn = wave_max(fabsf(d)), xn = wave_max(fabsf(x.hi));
      const bool stop = !(dn > tol * xn) || !(dn < 0.5f * prev);
      prev = dn;
      if (stop) break;
    }
    return x;
  }

  // the same for two right-hand sides, sharing the sweeps over A and L; a solution
  // whose corrections have stopped is left as it is while the other goes on
  __device__ __forceinline__ void refined_solve2(ff rhs0, ff rhs1, float tol, ff& x0, ff& x1) const {
    const bool mine = lane < m;
    {
      float y0, y1, z0, z1;
      forward2(mine ? rhs0.hi : 0.f, mine ? rhs1.hi : 0.f, y0, y1);
      backward2(y0, y1, z0, z1);
      x0 = ff{z0, 0.f};
      x1 = ff{z1, 0.f};
    }
    float prev0 = INFINITY, prev1 = INFINITY;
    bool run0 = true, run1 = true;
    for (int it = 0; it < REFINE_MAX && (run0 || run1); ++it) {
      S.vh[lane] = x0.hi;
      S.vl[lane] = x0.lo;
      S.wh[lane] = x1.hi;
      S.wl[lane] = x1.lo;
      wave_lds_sync();
      const ff r0 = residual(rhs0, S.vh, S.vl);
      const ff r1 = residual(rhs1, S.wh, S.wl);
      wave_lds_sync();
      float y0, y1, d0, d1;
      forward2(mine ? r0.hi + r0.lo : 0.f, mine ? r1.hi + r1.lo : 0.f, y0, y1);
      backward2(y0, y1, d0, d1);
      if (run0) {
        x0 = ff_add(x0, ff{d0, 0.f});
        const float dn = wave_max(fabsf(d0)), xn = wave_max(fabsf(x0.hi));
        run0 = dn > tol * xn && dn < 0.5f * prev0;
        prev0 = dn;
      }
      if (run1) {
        x1 = ff_add(x1, ff{d1, 0.f});
        const float dn = wave_max(fabsf(d1)), xn = wave_max(fabsf(x1.hi));
        run1 = dn > tol * xn && dn < 0.5f * prev1;
        prev1 = dn;
      }
    }
  }
};

// Fit cell c with one wave; returns true when it must be refitted in FP64.
template <int MB, bool MATERN>
__device__ __forceinline__ bool fit32_wave(const FitArgs& A, int c, WaveFitLds<MB>& S) {
  const int b = A.offsets[c], m = A.offsets[c + 1] - b;
  WaveFit<MB, MATERN> W(S, m);
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
  // A = K + Sigma, row `lane`, float-float; the identity past m
  const ff inv2l2{A.inv2l2_ff[0], A.inv2l2_ff[1]};
  const ff mc{A.mc_ff[0], A.mc_ff[1]};
  static_for<0, MB>([&](auto K) {
    constexpr int k = K;
    ff v{lane == k ? 1.f : 0.f, 0.f};
    if (k < m) {   // uniform
      const ff r2 = W.dist2(xh, xl, k);
      ff kv;
      if constexpr (MATERN) {
        const ff t = ff_mul(ff_sqrt(r2), mc);
        kv = ff_mul(ff_add(ff{1.f, 0.f}, t), ff_exp_neg_lean(t));
      } else {
        kv = ff_exp_neg_lean(ff_mul(r2, inv2l2));
      }
      if (k == lane) kv = ff_add(kv, ff{svh, svl});
      if (mine) v = kv;
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
        static_for<(j + 1) / 4, MB / 4>([&](auto G) {
          constexpr int g = G;
          const float4 cv = reinterpret_cast<const float4*>(S.col)[g];
          if constexpr (4 * g > j) W.Lr[4 * g] = fmaf(-l, cv.x, W.Lr[4 * g]);
          if constexpr (4 * g + 1 > j) W.Lr[4 * g + 1] = fmaf(-l, cv.y, W.Lr[4 * g + 1]);
          if constexpr (4 * g + 2 > j) W.Lr[4 * g + 2] = fmaf(-l, cv.z, W.Lr[4 * g + 2]);
          if constexpr (4 * g + 3 > j) W.Lr[4 * g + 3] = fmaf(-l, cv.w, W.Lr[4 * g + 3]);
        });
        wave_lds_sync();
      }
    }
  });
  // the packed factor (reciprocal diagonal) for the L^T solves and the store
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
      // c^2 r_ik^2 exp(-c r_ik) / l (Matern 3/2), a compensated sum over the row;
      // xi_s = A^{-1} a
      S.vh[lane] = a.hi;
      S.vl[lane] = a.lo;
      wave_lds_sync();
      const ff il = MATERN ? ff{A.inv_l_ff[0], A.inv_l_ff[1]} : ff{A.inv_l3_ff[0], A.inv_l3_ff[1]};
      const ff mc2{A.mc2_ff[0], A.mc2_ff[1]};
      const float il3f = A.inv_l3_ff[0];
      float gs = 0.f, gc = 0.f;   // minus the row sum, as Dot2 accumulators
      float* Drow = A.D32 ? A.D32 + A.loff[c] + (mine ? pk(lane, 0) : 0) : nullptr;
      static_for<0, MB>([&](auto K) {
        constexpr int k = K;
        if (k < m) {   // uniform; the diagonal term is zero (r = 0)
          const ff r2 = W.dist2(xh, xl, k);
          ff dk;
          if constexpr (MATERN) dk = ff_mul(ff_mul(ff_exp_neg_lean(ff_mul(ff_sqrt(r2), mc)), r2), mc2);
          else dk = ff_mul(ff{W.ah[k], W.al[k]}, r2);
          if (k == lane) dk = ff{0.f, 0.f};
          dot2_sub(gs, gc, dk.hi, dk.lo, S.vh[k], S.vl[k]);
          if (Drow && mine && k < lane)
            Drow[k] = MATERN ? A.mc2_ff[0] * r2.hi * expf(-A.mc_ff[0] * sqrtf(r2.hi)) * A.inv_l_ff[0]
                             : W.ah[k] * r2.hi * il3f;
        }
      });
      if (Drow && mine) Drow[lane] = 0.f;
      wave_lds_sync();
      const ff g = ff_mul(ff_neg(ff_two_sum(gs, gc)), il);
      ff xil, xis{0.f, 0.f};
      if (!A.svar) W.refined_solve2(mine ? g : ff{0.f, 0.f}, a, REFINE_TOL_ADJOINT, xil, xis);
      else xil = W.refined_solve(mine ? g : ff{0.f, 0.f}, REFINE_TOL_ADJOINT);
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
  // the per-cell store: (p, a) with low parts, sigma^2, the factor rows (copied from
  // LDS in store order, so consecutive lanes write consecutive floats; identity rows
  // for a cell left to the FP64 refit), box and A+
  if (mine) {
    reinterpret_cast<float4*>(A.ps32)[b + lane] = make_float4(xh[0], xh[1], xh[2], need64 ? 0.f : a.hi);
    reinterpret_cast<float4*>(A.plo32)[b + lane] = make_float4(xl[0], xl[1], xl[2], need64 ? 0.f : a.lo);
    A.sv32[b + lane] = svh;
  }
  {
    float* Lc = A.L32 + A.loff[c];
    const int np = m * (m + 1) / 2;
    for (int e = lane; e < np; e += 64) Lc[e] = need64 ? (packed_diag(e) ? 1.f : 0.f) : S.L[e];
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
