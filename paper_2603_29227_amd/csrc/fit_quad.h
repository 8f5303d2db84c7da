// One-workgroup FP32 fit of a cell with 64 < m <= 128 samples (Sec. IV-B.1, eq.
// log_gp_posterior_mean): the computation of fit32_wave (float-float assembly of
// A = K + Sigma, FP32 Cholesky, condition estimate, a = A^{-1} 1 refined against the
// float-float A, the adjoint vectors) for a 128 x 128 matrix held by four waves in
// 64 x 64 blocks.  Wave w owns rows 64 (w & 1) + lane and columns 64 (w >> 1) + k of
// A (float-float, in registers), so the blocks are A11 (wave 0), A21 (wave 1), A12
// (wave 2) and A22 (wave 3).  The blocked factorisation:
//   * wave 0 factors A11 = L11 L11^T in registers (right-looking by columns, as the
//     one-wave fit) and publishes L11 in the packed factor in LDS;
//   * wave 1 forms L21 = A21 L11^-T row by row in registers (a triangular solve per
//     lane against L11's broadcast rows);
//   * wave 3 forms the trailing update S = L21 L21^T on the matrix cores (three 32 x 32
//     tiles of v_mfma_f32_32x32x2f32 over k = 64, the lower triangle only), then
//     factors A22 - S = L22 L22^T in registers.
// Solves run on the packed factor in LDS in three hand-offs: wave 0 solves with L11,
// wave 1 applies L21 and solves with L22 (and back with L22^T), wave 0 applies L21^T
// and solves with L11^T.  Residuals b - A x and the adjoint sums are Dot2 partial
// sums per column block, combined by the waves of the first block.  Rows past m are
// the identity.
#pragma once

#include "fit_wave.h"

namespace ksdf {
namespace {

constexpr int QF_NP = 128 * 129 / 2;
typedef float qf_acc16 __attribute__((ext_vector_type(16)));

struct QuadFitLds {
  float4 xh[128];                 // cell-local coordinates (hi) and sigma^2 (hi)
  float4 xl[128];                 // their low parts
  alignas(16) float vh[128];      // float-float vectors broadcast to every wave
  alignas(16) float vl[128];
  alignas(16) float wh[128];
  alignas(16) float wl[128];
  alignas(16) float y[128];       // hand-offs of the triangular solves
  alignas(16) float col[64];      // the column of a register factorisation step
  float ps[2][128];               // partial sums of the second column block: [rhs][row]
  float pc[2][128];
  float red[2];                   // cross-wave reductions
  float red3[2][3];
  int flag;                       // 0 once a pivot failed
  alignas(16) float L[QF_NP + 64];   // packed factor rows, reciprocal diagonal (+ reach)
  float Alo[QF_NP + 256];         // low parts of A, packed lower triangle (A is symmetric),
                                  // then one dummy slot per thread
};

__device__ __forceinline__ int pkq(int i, int k) { return i * (i + 1) / 2 + k; }

template <bool MATERN>
struct QuadFit {
  QuadFitLds& S;
  int w, lane, rb, cb, R, m;
  float ah[64];           // row R of A, columns 64 cb + k (leading parts); identity past m
  float rd;               // 1 / L_RR for the lanes of waves 0 and 1

  // the low part of A[R][64 cb + k] from the packed lower triangle in LDS: entry
  // (max(R, C), min(R, C)), so the block below the diagonal reads its own rows and the
  // block above reads by column (consecutive lanes, consecutive entries)
  // (Rv: the row, passed through an empty asm so that the 64 addresses are formed at
  // each use instead of being kept live across the refinement loop)
  __device__ __forceinline__ float alo(int k, int Rv) const {
    const int C = 64 * cb + k;
    const int hi = max(C, Rv), lo = min(C, Rv);   // one branch-free form for every block
    return S.Alo[pkq(hi, 0) + lo];
  }

  __device__ __forceinline__ QuadFit(QuadFitLds& s, int m_)
      : S(s), w(threadIdx.x >> 6), lane(threadIdx.x & 63), rb(w & 1), cb(w >> 1),
        R(64 * rb + lane), m(m_), rd(1.f) {}

  // sum / max of a per-row value held by waves 0 and 1, to every thread
  __device__ __forceinline__ float rows_sum(float v) {
    __syncthreads();
    if (w < 2) {
      const float t = wave_sum(v);
      if (lane == 0) S.red[w] = t;
    }
    __syncthreads();
    return S.red[0] + S.red[1];
  }
  // three sums / two maxima with one pair of barriers
  __device__ __forceinline__ float3 rows_sum3(float a, float b, float c) {
    __syncthreads();
    if (w < 2) {
      const float ta = wave_sum(a), tb = wave_sum(b), tc = wave_sum(c);
      if (lane == 0) {
        S.red3[w][0] = ta;
        S.red3[w][1] = tb;
        S.red3[w][2] = tc;
      }
    }
    __syncthreads();
    return make_float3(S.red3[0][0] + S.red3[1][0], S.red3[0][1] + S.red3[1][1],
                       S.red3[0][2] + S.red3[1][2]);
  }
  __device__ __forceinline__ float2 rows_max2(float a, float b) {
    __syncthreads();
    if (w < 2) {
      const float ta = wave_max(a), tb = wave_max(b);
      if (lane == 0) {
        S.red3[w][0] = ta;
        S.red3[w][1] = tb;
      }
    }
    __syncthreads();
    return make_float2(fmaxf(S.red3[0][0], S.red3[1][0]), fmaxf(S.red3[0][1], S.red3[1][1]));
  }
  __device__ __forceinline__ float rows_max(float v) {
    __syncthreads();
    if (w < 2) {
      const float t = wave_max(v);
      if (lane == 0) S.red[w] = t;
    }
    __syncthreads();
    return fmaxf(S.red[0], S.red[1]);
  }

  // The triangular solves index no register array, so they run as loops (j uniform,
  // v_readlane with a scalar lane index) rather than unrolled: that keeps the
  // registers for the rows of A.
  // L y = b (b and y on the lanes of waves 0 and 1, rows R)
  __device__ __forceinline__ float forward(float b) {
    float y = 0.f;
    if (w == 0) {
      const float* row = S.L + pkq(lane, 0);
      float r = b;
#pragma unroll 4
      for (int j = 0; j < 64; ++j) {
        const float yj = readlane(r * rd, j);
        if (lane == j) y = yj;
        r = fmaf(-row[j], yj, r);
      }
      S.y[lane] = y;
    }
    __syncthreads();
    if (w == 1) {
      const float* row = S.L + pkq(64 + lane, 0);
      float r = b;
#pragma unroll 8
      for (int j = 0; j < 64; ++j) r = fmaf(-row[j], S.y[j], r);
#pragma unroll 4
      for (int j = 0; j < m - 64; ++j) {
        const float yj = readlane(r * rd, j);
        if (lane == j) y = yj;
        r = fmaf(-row[64 + j], yj, r);
      }
    }
    return y;
  }

  // L^T x = y
  __device__ __forceinline__ float backward(float y) {
    float x = 0.f;
    if (w == 1) {
      float r = y;
#pragma unroll 4
      for (int i = m - 65; i >= 0; --i) {
        const float xi = readlane(r * rd, i);
        if (lane == i) x = xi;
        r = fmaf(-S.L[pkq(64 + i, 64) + lane], xi, r);
      }
      S.y[64 + lane] = x;
    }
    __syncthreads();
    if (w == 0) {
      float r = y;
#pragma unroll 8
      for (int i = 0; i < 64; ++i) r = fmaf(-S.L[pkq(64 + i, 0) + lane], S.y[64 + i], r);
#pragma unroll 4
      for (int i = 63; i >= 0; --i) {
        const float xi = readlane(r * rd, i);
        if (lane == i) x = xi;
        r = fmaf(-S.L[pkq(i, 0) + lane], xi, r);
      }
    }
    __syncthreads();
    return x;
  }

  __device__ __forceinline__ float solve(float b) { return backward(forward(b)); }

  // (A x)_R with the FP32 leading parts (x on waves 0 and 1)
  __device__ __forceinline__ float matvec(float x) {
    if (w < 2) S.vh[R] = x;
    __syncthreads();
    float p = 0.f;
    static_for<0, 16>([&](auto G) {
      constexpr int g = G;
      const float4 v = reinterpret_cast<const float4*>(S.vh + 64 * cb)[g];
      p = fmaf(ah[4 * g], v.x, p);
      p = fmaf(ah[4 * g + 1], v.y, p);
      p = fmaf(ah[4 * g + 2], v.z, p);
      p = fmaf(ah[4 * g + 3], v.w, p);
    });
    if (w >= 2) S.ps[0][R] = p;
    __syncthreads();
    return w < 2 ? p + S.ps[0][R] : 0.f;
  }

  // Dot2 partial of -(A x) over this wave's columns for the float-float x in (vh, vl)
  __device__ __forceinline__ void partial(const float* vh, const float* vl, float& s, float& c) const {
    int Rv = R;
    asm volatile("" : "+v"(Rv));
    s = 0.f;
    c = 0.f;
    static_for<0, 16>([&](auto G) {
      constexpr int g = G;
      const float4 h = reinterpret_cast<const float4*>(vh + 64 * cb)[g];
      const float4 l = reinterpret_cast<const float4*>(vl + 64 * cb)[g];
      dot2_sub(s, c, ah[4 * g], alo(4 * g, Rv), h.x, l.x);
      dot2_sub(s, c, ah[4 * g + 1], alo(4 * g + 1, Rv), h.y, l.y);
      dot2_sub(s, c, ah[4 * g + 2], alo(4 * g + 2, Rv), h.z, l.z);
      dot2_sub(s, c, ah[4 * g + 3], alo(4 * g + 3, Rv), h.w, l.w);
      // keep the scheduler from hoisting every group's loads at once (registers)
      __builtin_amdgcn_sched_barrier(0);
    });
  }

  // rhs + own partial + the second column block's partial, as a float pair
  __device__ __forceinline__ ff combine(ff rhs, float s, float c, int k) const {
    const ff a = ff_two_sum(s, S.ps[k][R]);
    const ff h = ff_two_sum(rhs.hi, a.hi);
    return ff_fast_two_sum(h.hi, ((rhs.lo + c) + (S.pc[k][R] + a.lo)) + h.lo);
  }

  // rhs - (A x)_R in float-float (x on waves 0 and 1)
  __device__ __forceinline__ ff residual(ff rhs, ff x) {
    if (w < 2) {
      S.vh[R] = x.hi;
      S.vl[R] = x.lo;
    }
    __syncthreads();
    float s, c;
    partial(S.vh, S.vl, s, c);
    if (w >= 2) {
      S.ps[0][R] = s;
      S.pc[0][R] = c;
    }
    __syncthreads();
    return w < 2 ? combine(rhs, s, c, 0) : ff{0.f, 0.f};
  }
  __device__ __forceinline__ ff refined_solve(ff rhs, float tol) {
    const bool mine = w < 2 && R < m;
    ff x{solve(mine ? rhs.hi : 0.f), 0.f};
    float prev = INFINITY;
    for (int it = 0; it < REFINE_MAX; ++it) {
      const ff r = residual(rhs, x);
      const float d = solve(mine ? r.hi + r.lo : 0.f);
      x = ff_add(x, ff{d, 0.f});
      const float2 mx = rows_max2(fabsf(d), fabsf(x.hi));
      const float dn = mx.x, xn = mx.y;
      const bool stop = !(dn > tol * xn) || !(dn < 0.5f * prev);
      prev = dn;
      if (stop) break;
    }
    return x;
  }

  // squared distance of samples R and C, float-float
  __device__ __forceinline__ ff dist2(const float xh_[3], const float xl_[3], int C) const {
    const float4 h = S.xh[C], l = S.xl[C];
    return ff_norm2_lean(ff_sub_lean(xh_[0], xl_[0], h.x, l.x), ff_sub_lean(xh_[1], xl_[1], h.y, l.y),
                         ff_sub_lean(xh_[2], xl_[2], h.z, l.z));
  }
};

// Register Cholesky of a 64 x 64 block held one row per lane (Lr), first n columns
// (the rest identity); leaves 1 / L_ii in rd.  false on a non-positive pivot.
__device__ __forceinline__ bool block_chol64(float (&Lr)[64], float& rd, float* col, int n) {
  const int lane = threadIdx.x & 63;
  bool ok = true;
  rd = 1.f;
  static_for<0, 64>([&](auto J) {
    constexpr int j = J;
    if (ok && j < n) {
      const float d = readlane(Lr[j], j);
      if (!(d > 0.f)) {
        ok = false;
      } else {
        const float ljj = sqrtf(d), inv = 1.f / ljj;
        const float l = lane > j ? Lr[j] * inv : (lane == j ? ljj : 0.f);
        Lr[j] = l;
        if (lane == j) rd = inv;
        col[lane] = l;
        wave_lds_sync();
        static_for<(j + 1) / 4, 16>([&](auto G) {
          constexpr int g = G;
          const float4 cv = reinterpret_cast<const float4*>(col)[g];
          if constexpr (4 * g > j) Lr[4 * g] = fmaf(-l, cv.x, Lr[4 * g]);
          if constexpr (4 * g + 1 > j) Lr[4 * g + 1] = fmaf(-l, cv.y, Lr[4 * g + 1]);
          if constexpr (4 * g + 2 > j) Lr[4 * g + 2] = fmaf(-l, cv.z, Lr[4 * g + 2]);
          if constexpr (4 * g + 3 > j) Lr[4 * g + 3] = fmaf(-l, cv.w, Lr[4 * g + 3]);
        });
        wave_lds_sync();
      }
    }
  });
  return ok;
}

// Fit cell c (64 < m <= 128) with the whole workgroup; true when it must be refitted
// in FP64.
template <bool MATERN>
__device__ __forceinline__ bool fit32_quad(const FitArgs& A, int c, QuadFitLds& S) {
  const int b = A.offsets[c], m = A.offsets[c + 1] - b;
  QuadFit<MATERN> Q(S, m);
  const int w = Q.w, lane = Q.lane, cb = Q.cb, R = Q.R;
  const bool mine = R < m;
  // gather (waves 0 and 1): cell-local coordinates, exact as float-float
  if (w < 2) {
    float xh[3] = {0.f, 0.f, 0.f}, xl[3] = {0.f, 0.f, 0.f}, svh = 0.f, svl = 0.f;
    if (mine) {
      const long s = A.samples[b + R];
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
    S.xh[R] = make_float4(xh[0], xh[1], xh[2], svh);
    S.xl[R] = make_float4(xl[0], xl[1], xl[2], svl);
  }
  if (threadIdx.x == 0) S.flag = 1;
  __syncthreads();
  float xh[3], xl[3], svh, svl;
  {
    const float4 h = S.xh[R], l = S.xl[R];
    xh[0] = h.x; xh[1] = h.y; xh[2] = h.z; svh = h.w;
    xl[0] = l.x; xl[1] = l.y; xl[2] = l.z; svl = l.w;
  }
  // this wave's block of A = K + Sigma, float-float; the identity past m
  const ff inv2l2{A.inv2l2_ff[0], A.inv2l2_ff[1]};
  const ff mc{A.mc_ff[0], A.mc_ff[1]};
  float Lr[64];
  static_for<0, 64>([&](auto K) {
    constexpr int k = K;
    const int C = 64 * cb + k;
    ff v{R == C ? 1.f : 0.f, 0.f};
    if (C < m) {   // uniform
      const ff r2 = Q.dist2(xh, xl, C);
      ff kv;
      if constexpr (MATERN) {
        const ff t = ff_mul(ff_sqrt(r2), mc);
        kv = ff_mul(ff_add(ff{1.f, 0.f}, t), ff_exp_neg_lean(t));
      } else {
        kv = ff_exp_neg_lean(ff_mul(r2, inv2l2));
      }
      if (R == C) kv = ff_add(kv, ff{svh, svl});
      if (mine) v = kv;
    }
    Q.ah[k] = v.hi;
    // the lower triangle, each entry once (entries above it go to a per-lane dummy slot,
    // which keeps the store unconditional)
    S.Alo[C <= R ? pkq(R, 0) + C : QF_NP + threadIdx.x] = v.lo;
    Lr[k] = v.hi;
    __builtin_amdgcn_sched_barrier(0);   // one entry's temporaries at a time
  });
  // L11 (wave 0)
  if (w == 0) {
    float rd0;
    const bool ok = block_chol64(Lr, rd0, S.col, 64);
    if (ok) {
      static_for<0, 64>([&](auto K) {
        if (K < lane) S.L[pkq(lane, K)] = Lr[K];
      });
      S.L[pkq(lane, lane)] = rd0;
    } else if (lane == 0) {
      S.flag = 0;
    }
    Q.rd = rd0;
  }
  __syncthreads();
  bool ok = S.flag != 0;
  // L21 = A21 L11^-T (wave 1): each lane solves its row against L11, left-looking:
  // x_j = (a_j - sum_{k<j} x_k L11[j][k]) / L11[j][j] with row j of L11 read by
  // broadcast loads (contiguous, so pairs merge) and four partial sums per row
  if (ok && w == 1) {
    static_for<0, 64>([&](auto J) {
      constexpr int j = J;
      const float* Lj = S.L + pkq(j, 0);
      float t[4] = {Lr[j], 0.f, 0.f, 0.f};
      static_for<0, j>([&](auto K) {
        constexpr int k = K;
        t[k % 4] = fmaf(-Lr[k], Lj[k], t[k % 4]);
      });
      Lr[j] = ((t[0] + t[1]) + (t[2] + t[3])) * Lj[j];   // Lj[j]: the reciprocal diagonal
    });
    static_for<0, 64>([&](auto K) { S.L[pkq(64 + lane, K)] = Lr[K]; });
  }
  __syncthreads();
  // A22 - L21 L21^T = L22 L22^T (wave 3; the trailing update on the matrix cores)
  if (ok && w == 3) {
    // lane l supplies A[l mod 32][l div 32] and B[l div 32][l mod 32] of each k-step
    // and receives D[8 (r div 4) + 4 (l div 32) + r mod 4][l mod 32] in register r
    const int hi = lane >> 5, lo = lane & 31;
    // tiles (I, J) = (0, 0), (1, 0), (1, 1) one after the other: rows 32 I.. of L21
    // times rows 32 J.. transposed; the lower triangle of S goes into the rows of L22
    // (read back below, then overwritten by the factor).  Every tile's operands are read
    // before any tile is stored: L21 and the L22 rows do not overlap.
    static_for<0, 3>([&](auto TI) {
      constexpr int ti = TI;
      constexpr int I = ti == 0 ? 0 : 1, J = ti == 2 ? 1 : 0;
      qf_acc16 acc = {};
      static_for<0, 32>([&](auto T) {
        constexpr int t = T;
        const float xa = S.L[pkq(64 + 32 * I + lo, 2 * t + hi)];
        const float xb = S.L[pkq(64 + 32 * J + lo, 2 * t + hi)];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(xa, xb, acc, 0, 0, 0);
        if constexpr (t % 4 == 3) __builtin_amdgcn_sched_barrier(0);
      });
      __builtin_amdgcn_sched_barrier(0);
      static_for<0, 16>([&](auto Rg) {
        constexpr int r = Rg;
        const int row = 32 * I + 8 * (r / 4) + 4 * hi + r % 4, colj = 32 * J + lo;
        if (colj <= row) S.L[pkq(64 + row, 64 + colj)] = acc[r];
      });
    });
    wave_lds_sync();
    static_for<0, 64>([&](auto K) {
      if (K <= lane) Lr[K] -= S.L[pkq(64 + lane, 64 + K)];
    });
    wave_lds_sync();
    float rd3;
    const bool ok3 = block_chol64(Lr, rd3, S.col, m - 64);
    if (ok3) {
      static_for<0, 64>([&](auto K) {
        if (K < lane) S.L[pkq(64 + lane, 64 + K)] = Lr[K];
      });
      S.L[pkq(64 + lane, 64 + lane)] = rd3;
    } else if (lane == 0) {
      S.flag = 0;
    }
  }
  __syncthreads();
  ok = S.flag != 0;
  if (w == 1) Q.rd = S.L[pkq(64 + lane, 64 + lane)];
  float cond = INFINITY;
  if (ok) {
    // lambda_max by power iteration (ones start), lambda_min by inverse iteration
    // (alternating-sign start), as the one-wave fit
    const bool row = w < 2 && mine;
    float x = row ? 1.f : 0.f, lmax = 0.f;
    for (int it = 0; it < 4; ++it) {
      const float y = Q.matvec(x);
      const float3 r3 = Q.rows_sum3(x * x, x * y, y * y);
      lmax = r3.y / r3.x;
      x = y / sqrtf(r3.z);
    }
    // inverse iteration: |x| = sqrt(m) at the start, 1 after each normalisation
    x = row ? ((R & 1) ? -1.f : 1.f) : 0.f;
    float nx = sqrtf((float)m), inv_lmin = 0.f;
    for (int it = 0; it < 4; ++it) {
      const float y = Q.solve(x);
      const float ny = sqrtf(Q.rows_sum(y * y));
      inv_lmin = ny / nx;
      x = y / ny;
      nx = 1.f;
    }
    cond = lmax * inv_lmin;
  }
  const bool need64 = !ok || !(cond <= (float)A.cond_thr);
  const bool row = w < 2 && mine;
  ff a{0.f, 0.f};
  if (!need64) {
    a = Q.refined_solve(ff{row ? 1.f : 0.f, 0.f}, REFINE_TOL);
    if (!row) a = ff{0.f, 0.f};
    if (A.adjoint) {
      // xi_l = A^{-1} (dA/dl) a, a Dot2 sum over each column block; xi_s = A^{-1} a
      if (w < 2) {
        S.vh[R] = a.hi;
        S.vl[R] = a.lo;
      }
      __syncthreads();
      const ff il = MATERN ? ff{A.inv_l_ff[0], A.inv_l_ff[1]} : ff{A.inv_l3_ff[0], A.inv_l3_ff[1]};
      const ff mc2{A.mc2_ff[0], A.mc2_ff[1]};
      const float il3f = A.inv_l3_ff[0];
      float gs = 0.f, gc = 0.f;
      float* Drow = (A.D32 && mine) ? A.D32 + A.loff[c] + pkq(R, 0) : nullptr;
      static_for<0, 64>([&](auto K) {
        constexpr int k = K;
        const int C = 64 * cb + k;
        if (C < m) {   // uniform; the diagonal term is zero (r = 0)
          const ff r2 = Q.dist2(xh, xl, C);
          ff dk;
          if constexpr (MATERN) dk = ff_mul(ff_mul(ff_exp_neg_lean(ff_mul(ff_sqrt(r2), mc)), r2), mc2);
          else dk = ff_mul(ff{Q.ah[k], Q.alo(k, R)}, r2);
          if (C == R) dk = ff{0.f, 0.f};
          dot2_sub(gs, gc, dk.hi, dk.lo, S.vh[C], S.vl[C]);
          if (Drow && C < R)
            Drow[C] = MATERN ? A.mc2_ff[0] * r2.hi * expf(-A.mc_ff[0] * sqrtf(r2.hi)) * A.inv_l_ff[0]
                             : Q.ah[k] * r2.hi * il3f;
        }
        __builtin_amdgcn_sched_barrier(0);
      });
      if (Drow && w < 2) Drow[R] = 0.f;
      if (w >= 2) {
        S.ps[0][R] = gs;
        S.pc[0][R] = gc;
      }
      __syncthreads();
      ff g{0.f, 0.f};
      if (w < 2) g = ff_mul(ff_neg(Q.combine(ff{0.f, 0.f}, gs, gc, 0)), il);
      __syncthreads();
      ff xil, xis{0.f, 0.f};
      // one right-hand side at a time: the two-RHS sweep needs more registers than the
      // four-wave layout leaves
      xil = Q.refined_solve(row ? g : ff{0.f, 0.f}, REFINE_TOL_ADJOINT);
      if (!A.svar) xis = Q.refined_solve(a, REFINE_TOL_ADJOINT);
      if (row) {
        float4 xv;
        xv.x = xil.hi;
        xv.y = A.svar ? 0.f : xis.hi;
        xv.z = xil.lo;
        xv.w = A.svar ? 0.f : xis.lo;
        reinterpret_cast<float4*>(A.xi32)[b + R] = xv;
      }
    }
  }
  // the per-cell store
  if (row) {
    reinterpret_cast<float4*>(A.ps32)[b + R] = make_float4(xh[0], xh[1], xh[2], need64 ? 0.f : a.hi);
    reinterpret_cast<float4*>(A.plo32)[b + R] = make_float4(xl[0], xl[1], xl[2], need64 ? 0.f : a.lo);
    A.sv32[b + R] = svh;
  }
  {
    float* Lc = A.L32 + A.loff[c];
    const int np = m * (m + 1) / 2;
    for (int e = threadIdx.x; e < np; e += 256) Lc[e] = need64 ? (packed_diag(e) ? 1.f : 0.f) : S.L[e];
  }
  const float apos = Q.rows_sum(row && !need64 ? fmaxf(a.hi, 0.f) : 0.f);
  float lo3[3], hi3[3];
  for (int d = 0; d < 3; ++d) {
    lo3[d] = -Q.rows_max(row ? -xh[d] : -1e30f);
    hi3[d] = Q.rows_max(row ? xh[d] : -1e30f);
  }
  if (threadIdx.x == 0) {
    float* box = A.box32 + 8L * c;
    box[0] = lo3[0]; box[1] = lo3[1]; box[2] = lo3[2];
    box[3] = apos;
    box[4] = hi3[0]; box[5] = hi3[1]; box[6] = hi3[2];
    box[7] = 0.f;
    A.cond32[c] = cond;
    A.cstatus[c] = 0;
    if (A.user_status && !need64) A.user_status[c] = 0;
  }
  return need64;
}

}  // namespace
}  // namespace ksdf
