// Float-float ("double-single") arithmetic on FP32 instructions.
//
// A value is the unevaluated sum hi + lo of two floats with |lo| <= ulp(hi)/2,
// about 44 significant bits.  The error-free transformations are the classical
// ones: Knuth's TwoSum, Dekker's Fast2Sum, and the FMA-based TwoProduct
// (Dekker 1971; Knuth, TAOCP vol. 2, sec. 4.2.2).  Contraction is disabled in this
// header so the compiler cannot fuse the steps that carry the rounding errors.
#pragma once

#include <hip/hip_runtime.h>

namespace ksdf {

struct ff {
  float hi, lo;
};

__host__ __device__ __forceinline__ ff ff_two_sum(float a, float b) {
#pragma clang fp contract(off)
  const float s = a + b;
  const float bb = s - a;
  const float e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

__host__ __device__ __forceinline__ ff ff_fast_two_sum(float a, float b) {  // |a| >= |b|
#pragma clang fp contract(off)
  const float s = a + b;
  return {s, b - (s - a)};
}

__host__ __device__ __forceinline__ ff ff_two_prod(float a, float b) {
#pragma clang fp contract(off)
  const float p = a * b;
  return {p, __builtin_fmaf(a, b, -p)};
}

__host__ __device__ __forceinline__ ff ff_add(ff a, ff b) {
#pragma clang fp contract(off)
  ff s = ff_two_sum(a.hi, b.hi);
  const ff t = ff_two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = ff_fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return ff_fast_two_sum(s.hi, s.lo);
}

__host__ __device__ __forceinline__ ff ff_neg(ff a) { return {-a.hi, -a.lo}; }

__host__ __device__ __forceinline__ ff ff_mul(ff a, ff b) {
#pragma clang fp contract(off)
  ff p = ff_two_prod(a.hi, b.hi);
  p.lo = __builtin_fmaf(a.hi, b.lo, p.lo);
  p.lo = __builtin_fmaf(a.lo, b.hi, p.lo);
  return ff_fast_two_sum(p.hi, p.lo);
}

__host__ __device__ __forceinline__ ff ff_mul_f(ff a, float b) {
#pragma clang fp contract(off)
  ff p = ff_two_prod(a.hi, b);
  p.lo = __builtin_fmaf(a.lo, b, p.lo);
  return ff_fast_two_sum(p.hi, p.lo);
}

// exp(-t) for t >= 0 in float-float.  Range reduction t = n ln2 + r with ln2 split
// into three floats (Cody-Waite; the first part has 16 significant bits so n*c1 is
// exact for n < 2^8), then the Taylor series of exp(-r), |r| <= ln2/2, to degree 13
// (truncation < 2e-17), then an exact scaling by 2^-n.
__host__ __device__ __forceinline__ ff ff_exp_neg(ff t) {
#pragma clang fp contract(off)
  constexpr double LN2 = 0.69314718055994530941723212145818;
  constexpr float C1 = 0.693145751953125f;
  constexpr float C2 = (float)(LN2 - (double)C1);
  constexpr float C3 = (float)(LN2 - (double)C1 - (double)C2);
  if (!(t.hi < 103.0f)) return {0.f, 0.f};
  const float n = rintf(t.hi * 1.44269504088896341f);
  ff r = ff_two_sum(t.hi - n * C1, t.lo);          // t.hi - n*C1 is exact (Sterbenz)
  r = ff_add(r, ff_neg(ff_two_prod(n, C2)));
  r = ff_add(r, ff{-n * C3, 0.f});
  const ff x = ff_neg(r);
  // Horner on 1/k!, k = 13..0, coefficients split to float-float at compile time
#define KSDF_INV_FACT(k, v) {(float)(v), (float)((v) - (double)(float)(v))}
  constexpr ff coef[14] = {
      KSDF_INV_FACT(0, 1.0), KSDF_INV_FACT(1, 1.0), KSDF_INV_FACT(2, 1.0 / 2),
      KSDF_INV_FACT(3, 1.0 / 6), KSDF_INV_FACT(4, 1.0 / 24), KSDF_INV_FACT(5, 1.0 / 120),
      KSDF_INV_FACT(6, 1.0 / 720), KSDF_INV_FACT(7, 1.0 / 5040), KSDF_INV_FACT(8, 1.0 / 40320),
      KSDF_INV_FACT(9, 1.0 / 362880), KSDF_INV_FACT(10, 1.0 / 3628800),
      KSDF_INV_FACT(11, 1.0 / 39916800), KSDF_INV_FACT(12, 1.0 / 479001600),
      KSDF_INV_FACT(13, 1.0 / 6227020800)};
#undef KSDF_INV_FACT
  ff p = coef[13];
#pragma unroll
  for (int k = 12; k >= 0; --k) p = ff_add(ff_mul(p, x), coef[k]);
  const int e = -(int)n;
  return {ldexpf(p.hi, e), ldexpf(p.lo, e)};
}

// Table-driven exp(-t), t >= 0, in float-float: t = k ln2/64 + r with |r| <= ln2/128,
// exp(-t) = 2^-(k/64) * exp(-r); 2^-(j/64) for j < 64 comes from a compile-time table
// (double-precision Taylor sums split into float pairs) and exp(-r) from its Taylor
// series to degree 6 (truncation below 1e-19).  ln2/64 is split into three floats,
// the first with 10 significant bits so k*C1 is exact for k < 2^14.
namespace exp_tab_detail {
constexpr double taylor_exp(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 40; ++k) {
    term *= x / k;
    sum += term;
  }
  return sum;
}
struct Tab {
  float hi[64], lo[64];
};
constexpr Tab make_tab() {
  Tab t{};
  for (int j = 0; j < 64; ++j) {
    const double v = taylor_exp(-0.69314718055994530942 * j / 64.0);
    t.hi[j] = (float)v;
    t.lo[j] = (float)(v - (double)(float)v);
  }
  return t;
}
}  // namespace exp_tab_detail

// The table in constant memory: a constexpr local indexed at run time would be copied
// into every lane's private memory.
static __constant__ const exp_tab_detail::Tab kExpTab = exp_tab_detail::make_tab();

__host__ __device__ __forceinline__ ff ff_exp_neg_tab(ff t) {
#pragma clang fp contract(off)
  const exp_tab_detail::Tab& TAB = kExpTab;
  constexpr float C1 = 0.0108184814453125f;
  constexpr float C2 = 1.1943250683543738e-05f;
  constexpr float C3 = 2.531013593154441e-13f;
  constexpr float INV = 92.33248261689366f;    // 64 / ln 2
  if (!(t.hi < 103.0f)) return {0.f, 0.f};
  const float k = rintf(t.hi * INV);
  ff r = ff_two_sum(t.hi - k * C1, t.lo);
  r = ff_add(r, ff_neg(ff_two_prod(k, C2)));
  r = ff_add(r, ff{-k * C3, 0.f});
  const ff x = ff_neg(r);
#define KSDF_C(v) ff{(float)(v), (float)((v) - (double)(float)(v))}
  ff p = KSDF_C(1.0 / 720);
  p = ff_add(ff_mul(p, x), KSDF_C(1.0 / 120));
  p = ff_add(ff_mul(p, x), KSDF_C(1.0 / 24));
  p = ff_add(ff_mul(p, x), KSDF_C(1.0 / 6));
  p = ff_add(ff_mul(p, x), KSDF_C(0.5));
  p = ff_add(ff_mul(p, x), ff{1.f, 0.f});
  p = ff_add(ff_mul(p, x), ff{1.f, 0.f});
#undef KSDF_C
  const int ki = (int)k;
  const int j = ki & 63;
  p = ff_mul(p, ff{TAB.hi[j], TAB.lo[j]});
  const int e = -(ki >> 6);
  return {ldexpf(p.hi, e), ldexpf(p.lo, e)};
}

// exp(-t), t >= 0, in float-float to a few parts in 1e14, cheaper than ff_exp_neg_tab:
// the same reduction (t = k ln2/64 + r, |r| <= ln2/128), then exp(-r) = 1 - r + r^2/2
// - r^3/6 + r^4/24 with 1 - r_hi exact as a float pair, r_hi^2/2 exact by TwoProduct,
// and -r_lo + r_hi r_lo - r^3/6 + r^4/24 (below 3e-8) in FP32, whose rounding (below
// 2e-15) and the dropped r^5/120 (below 4e-14) are the series' errors; then the table
// factor.
__host__ __device__ __forceinline__ ff ff_exp_neg_fast(ff t) {
#pragma clang fp contract(off)
  const exp_tab_detail::Tab& TAB = kExpTab;
  constexpr float C1 = 0.0108184814453125f;
  constexpr float C2 = 1.1943250683543738e-05f;
  constexpr float C3 = 2.531013593154441e-13f;
  constexpr float INV = 92.33248261689366f;    // 64 / ln 2
  if (!(t.hi < 103.0f)) return {0.f, 0.f};
  const float k = rintf(t.hi * INV);
  ff r = ff_two_sum(t.hi - k * C1, t.lo);
  r = ff_add(r, ff_neg(ff_two_prod(k, C2)));
  r = ff_add(r, ff{-k * C3, 0.f});
  const float rh = r.hi;
  // -r_lo + r_hi r_lo (the cross term of r^2 / 2) - r^3/6 + r^4/24
  const float rest = __builtin_fmaf(rh * rh * rh, __builtin_fmaf(rh, 1.f / 24, -1.f / 6),
                                    __builtin_fmaf(rh, r.lo, -r.lo));
  ff p = ff_two_sum(1.f, -rh);
  p = ff_add(p, ff_two_prod(rh, 0.5f * rh));
  p = ff_add(p, ff{rest, 0.f});
  const int ki = (int)k;
  const int j = ki & 63;
  p = ff_mul(p, ff{TAB.hi[j], TAB.lo[j]});
  const int e = -(ki >> 6);
  return {ldexpf(p.hi, e), ldexpf(p.lo, e)};
}

// exp(-t) for float-float t >= 0, the reduction and series of ff_exp_neg_fast with
// fewer operations: r = t - k ln2/64 from exact products (k C1, and TwoProduct for
// k C2) and one TwoSum, the series' leading terms 1 - r_hi (exact by Fast2Sum, as
// |r_hi| < 1/2) and r_hi^2/2 (exact by TwoProduct) added by Fast2Sum, the rest in
// FP32.  Below about 1e-13 relative for t < 87; 0 from t >= 87 (exp(-87) is at the
// bottom of the FP32 normal range).  Branch-free.
__host__ __device__ __forceinline__ ff ff_exp_neg_lean(ff t) {
#pragma clang fp contract(off)
  const exp_tab_detail::Tab& TAB = kExpTab;
  constexpr float C1 = 0.0108184814453125f;
  constexpr float C2 = 1.1943250683543738e-05f;
  constexpr float C3 = 2.531013593154441e-13f;
  constexpr float INV = 92.33248261689366f;    // 64 / ln 2
  const bool live = t.hi < 87.f;
  const float th = live ? t.hi : 0.f, tl = live ? t.lo : 0.f;
  const float k = rintf(th * INV);
  const float r0 = th - k * C1;                 // exact: k C1 has at most 24 bits, Sterbenz
  const ff p = ff_two_prod(k, C2);
  const ff r1 = ff_two_sum(r0, -p.hi);
  const ff r = ff_fast_two_sum(r1.hi, (__builtin_fmaf(-k, C3, tl - p.lo)) + r1.lo);
  const float rh = r.hi;
  const float rest = __builtin_fmaf(rh * rh * rh, __builtin_fmaf(rh, 1.f / 24, -1.f / 6),
                                    __builtin_fmaf(rh, r.lo, -r.lo));
  const ff a = ff_fast_two_sum(1.f, -rh);
  const ff q = ff_two_prod(rh, 0.5f * rh);
  const ff b = ff_fast_two_sum(a.hi, q.hi);
  ff e = ff_fast_two_sum(b.hi, ((a.lo + q.lo) + b.lo) + rest);
  const int ki = (int)k;
  const int j = ki & 63;
  e = ff_mul(e, ff{TAB.hi[j], TAB.lo[j]});
  const int sh = -(ki >> 6);
  return live ? ff{ldexpf(e.hi, sh), ldexpf(e.lo, sh)} : ff{0.f, 0.f};
}

// (xh + xl) - (yh + yl) for two float-float coordinates of the same frame: TwoSum of
// the leading parts and one rounding of the low parts' difference (below 2^-47 of the
// operands).
__host__ __device__ __forceinline__ ff ff_sub_lean(float xh, float xl, float yh, float yl) {
#pragma clang fp contract(off)
  const ff s = ff_two_sum(xh, -yh);
  return ff_fast_two_sum(s.hi, s.lo + (xl - yl));
}

// |v|^2 of a float-float 3-vector: the squares of the leading parts exact by
// TwoProduct and added by TwoSum, the cross terms 2 hi lo and every error term summed
// in FP32 (about 2^-46 relative; the dropped lo^2 are smaller still).
__host__ __device__ __forceinline__ ff ff_norm2_lean(ff x, ff y, ff z) {
#pragma clang fp contract(off)
  const ff px = ff_two_prod(x.hi, x.hi), py = ff_two_prod(y.hi, y.hi), pz = ff_two_prod(z.hi, z.hi);
  const ff s = ff_two_sum(px.hi, py.hi);
  const ff t = ff_two_sum(s.hi, pz.hi);
  float e = ((px.lo + py.lo) + (pz.lo + s.lo)) + t.lo;
  e = __builtin_fmaf(2.f * x.hi, x.lo, e);
  e = __builtin_fmaf(2.f * y.hi, y.lo, e);
  e = __builtin_fmaf(2.f * z.hi, z.lo, e);
  return ff_fast_two_sum(t.hi, e);
}

// One step of a compensated dot product (Ogita, Rump and Oishi's Dot2, with the
// float-float operands' cross terms): s + c -= (ah + al)(xh + xl), the product's
// rounding error (TwoProduct) and the sum's (TwoSum) collected in c, al xl dropped.
// The result is as accurate as if computed in twice the working precision.
__host__ __device__ __forceinline__ void dot2_sub(float& s, float& c, float ah, float al, float xh,
                                                  float xl) {
#pragma clang fp contract(off)
  const float p = ah * xh;
  const float pe = __builtin_fmaf(ah, xh, -p);
  const float t = s - p;
  const float bb = t - s;
  const float se = (s - (t - bb)) + (-p - bb);
  s = t;
  c = c + (se - pe);
  c = __builtin_fmaf(-ah, xl, c);
  c = __builtin_fmaf(-al, xh, c);
}

// Natural log of a float-float f > 0 to about 1e-13 absolute: the FP32 log y0 of the
// leading part corrected by ln g ~ g - 1 with g = f exp(-y0) = 1 + O(1e-7) (the
// dropped (g - 1)^2 / 2 is below 1e-14).  With w = exp(-|y0|) from the float-float
// exponential, g - 1 = f w - 1 for y0 >= 0 and (f - w) / w for y0 < 0.
__host__ __device__ __forceinline__ ff ff_log(ff f) {
#pragma clang fp contract(off)
  const float y0 = logf(f.hi);
  const ff w = ff_exp_neg_fast(ff{fabsf(y0), 0.f});
  float d;
  if (y0 >= 0.f) {
    const ff g1 = ff_add(ff_mul(f, w), ff{-1.f, 0.f});
    d = g1.hi + g1.lo;
  } else {
    const ff num = ff_add(f, ff_neg(w));
    d = (num.hi + num.lo) / w.hi;
  }
  return ff_two_sum(y0, d);
}

// Square root of a float-float a >= 0: the float root s of the leading part, then one
// Newton step on the exact residual a - s^2 (s^2 by TwoProduct), which doubles the
// number of correct bits.
__host__ __device__ __forceinline__ ff ff_sqrt(ff a) {
#pragma clang fp contract(off)
  if (!(a.hi > 0.f)) return {0.f, 0.f};
  const float s = sqrtf(a.hi);
  const ff r = ff_add(a, ff_neg(ff_two_prod(s, s)));
  return ff_fast_two_sum(s, r.hi / (2.f * s));
}

}  // namespace ksdf
