// Query backward: the vector-Jacobian product of ksdf_query (adjoint of Sec. IV-B).
//
// For a query x with argmin cell c (held fixed: the min-fusion is piecewise), scaled
// kernel values e_i = exp(-(z_i^2 - d^2)/2l^2), f' = sum a_i e_i, w' = sum a_i e_i d_i
// (d_i = x - x_i), the outputs and their derivatives are
//   u = sqrt(d^2 - 2 l^2 ln f')        du/dx = w'/(f' u),  du/dl = (u^2 - Z)/(l u),
//                                       du/da_i = -l^2 e_i/(u f'),  Z = sum a e z^2 / f'
//   g = w'/|w'|                        dg = (I - g g^T) dw'/|w'|,
//                                       dw'/dx = f' I - sum a e d d^T / l^2   (kernel Hessian)
//                                       dw'/dl = sum a e z^2 d / l^3,  dw'/da_i = e_i d_i
//   var = sum c_i^2 sigma_i^2          d var/d z_j = 2 alpha (-sigma_j^2 c_j (c_j + s_j)
//                                                   + s_j V + c_j P),  P = sum sigma^2 c s,
//                                       d var/d alpha = sum 2 sigma^2 c_i (s_i (h - z_i)(B_i + 1)
//                                                   - alpha s_i Var_s(z)),  B_i = alpha(h - z_i) + 1
//   var_f = 1 - k^T A^{-1} k           d/dx = (2/l^2) sum beta_i k_i d_i,  beta = A^{-1} k,
//                                       d/dl|_A = -2 sum beta k z^2 / l^3,  d/dA = beta beta^T.
// The fit enters through a = A^{-1} 1: for a weight cotangent abar, d/dtheta =
// -abar^T A^{-1} (dA/dtheta) a = -abar . xi_theta, with xi_l = A^{-1} (dA/dl) a and
// xi_s = A^{-1} a prepared per cell by the fit.  So every query's contribution to
// (dL/dl, dL/dsigma^2) is local; they are summed in a fixed order in FP64, which makes
// the hyperparameter gradient deterministic without atomics.  alpha = 1/(2 l^2) is
// differentiated through when tied.  k* is recomputed, never stored.
#include <cmath>

#include "ff.h"
#include "ksdf_internal.h"
#include "wave_ops.h"

namespace ksdf {
namespace {

constexpr int BT = 256;

template <class T>
struct BwdArgs {
  const T* __restrict__ pts;
  long Q;
  const int8_t* sign;
  const int* argmin;
  const T* d_mean;
  const T* d_grad;
  const T* d_var;
  const T* d_var_f;
  T* d_points;
  double* part;            // [Q,2] per-query (dL/dl, dL/dsigma^2)
  int n_cells;
  const int* offsets;
  const long* loff;
  const T* ps;             // [nnz,4] (px,py,pz,a) cell-local
  const float* plo;        // FP32 store: float-float low parts of ps
  const T* sv;
  const T* L;              // packed rows, reciprocal diagonal
  const T* xi;             // [nnz,2] (FP64) or [nnz+pad,4] float-float (FP32)
  const T* D;              // packed dA/dl or null
  const double* centre64;
  const float* box;        // [n,8] sample AABB (cell-local)
  T ell, two_l2, alpha;
  float c2_ff[2];          // log2(e) / (2 l^2) as a float pair (FP32 models)
  float mc_ff[2];          // Matern c = sqrt(3) / l and c log2(e) as float pairs
  float mcl_ff[2];
  double ell_d, alpha_d;   // the same in FP64
  int alpha_tied;
  int uniform_noise;
  // the softplus margin cost (ksdf_cost_backward): when c_mean is set, the mean and
  // var cotangents are formed from the forward outputs instead of read
  const T* c_mean;
  const T* c_var;
  T c_margin, c_kvar;
  T* c_cost;               // per-query cost, or null
};

// Cotangents of mean and var for query q: the given ones, or those of the cost
// softplus(t), t = margin - mean + kvar sqrt(var): d/dmean = -sigmoid(t) and
// d/dvar = kvar sigmoid(t) / (2 sqrt(var)), with the stable forms of sigmoid and
// softplus (max(t, 0) + log1p(e^-|t|)); var is clamped below at 1e-30.
template <class T>
__device__ __forceinline__ void mean_var_cotangents(const BwdArgs<T>& A, long q, T& gm, T& gv) {
  gm = A.d_mean ? A.d_mean[q] : T(0);
  gv = A.d_var ? A.d_var[q] : T(0);
  if (A.c_mean) {
    const T sd = sqrt(fmax(A.c_var[q], T(1e-30)));
    const T t = A.c_margin - A.c_mean[q] + A.c_kvar * sd;
    const T e = exp(-fabs(t));
    const T sg = t >= T(0) ? T(1) / (T(1) + e) : e / (T(1) + e);
    gm = -sg;
    gv = A.c_kvar * sg / (T(2) * sd);
    if (A.c_cost) A.c_cost[q] = fmax(t, T(0)) + log1p(e);
  }
}

template <class T>
__device__ __forceinline__ T aabb_d2(const float* bx, T x, T y, T z) {
  const T ex = fmax(fmax((T)bx[0] - x, T(0)), x - (T)bx[4]);
  const T ey = fmax(fmax((T)bx[1] - y, T(0)), y - (T)bx[5]);
  const T ez = fmax(fmax((T)bx[2] - z, T(0)), z - (T)bx[6]);
  return ex * ex + ey * ey + ez * ez;
}

// One query's VJP on its argmin cell, per-thread loops (the plain path; also the
// FP32 path, where the wave calls it with a wave-uniform cell so the per-cell data
// arrive through scalar loads).  With VARF (a var_f cotangent is given), v is
// per-thread storage for k, then L^{-1} k, then beta = A^{-1} k; without it the two
// triangular solves and v are not needed.
template <class T, bool VARF>
__device__ __forceinline__ void query_vjp(const BwdArgs<T>& A, long q, int c, T* v, T out_dx[3],
                                          double out_th[2]) {
  const T lt = A.ell;
  const T x0 = A.pts[3 * q], x1 = A.pts[3 * q + 1], x2 = A.pts[3 * q + 2];
  const T s = A.sign ? (T)A.sign[q] : T(1);
  T gm, gv;
  mean_var_cotangents(A, q, gm, gv);
  T gg[3] = {T(0), T(0), T(0)};
  if (A.d_grad)
    for (int d = 0; d < 3; ++d) gg[d] = A.d_grad[3 * q + d];
  const T gf = VARF && A.d_var_f ? A.d_var_f[q] : T(0);
  const int b = A.offsets[c], m = A.offsets[c + 1] - b;
  const T* p = A.ps + 4L * b;
  const T* sv = A.sv + b;
  const T* Lc = A.L + A.loff[c];
  constexpr int XS = sizeof(T) == 4 ? 4 : 2;   // FP32 store: float-float pairs, hi first
  const T* xi = A.xi + XS * (long)b;
  const double* cc = A.centre64 + 3L * c;
  const T l0 = x0 - (T)cc[0], l1 = x1 - (T)cc[1], l2 = x2 - (T)cc[2];
  const T inv2l2 = T(1) / A.two_l2;
  // scaling reference: the exact nearest sample (any reference gives the same result)
  T d2 = (T)INFINITY;
  for (int i = 0; i < m; ++i) {
    const T dx = l0 - p[4 * i], dy = l1 - p[4 * i + 1], dz = l2 - p[4 * i + 2];
    d2 = fmin(d2, dx * dx + dy * dy + dz * dz);
  }
  const T ginv = exp(-d2 * inv2l2);
  const T zmin = sqrt(d2);
  // pass A: f', w', Z, softmin moments, k
  T f = 0, w[3] = {0, 0, 0}, Za = 0, S = 0, M1 = 0, M2 = 0;
  for (int i = 0; i < m; ++i) {
    const T dx = l0 - p[4 * i], dy = l1 - p[4 * i + 1], dz = l2 - p[4 * i + 2];
    const T z2 = dx * dx + dy * dy + dz * dz;
    const T e = exp(-(z2 - d2) * inv2l2);
    const T ae = p[4 * i + 3] * e;
    f += ae;
    w[0] += ae * dx;
    w[1] += ae * dy;
    w[2] += ae * dz;
    Za += ae * z2;
    const T t = sqrt(z2) - zmin;
    const T sm = exp(-A.alpha * t);
    S += sm;
    M1 += sm * t;
    M2 += sm * t * t;
    if constexpr (VARF) v[i] = e * ginv;
  }
  T vv = 0;
  if constexpr (VARF) {
    // forward substitution: v <- L^{-1} k
    for (int i = 0; i < m; ++i) {
      const T* row = Lc + (long)i * (i + 1) / 2;
      T t = v[i];
      for (int j = 0; j < i; ++j) t -= row[j] * v[j];
      v[i] = t * row[i];
      vv += v[i] * v[i];
    }
    // backward substitution: v <- L^{-T} v = A^{-1} k (row-oriented, last row first)
    for (int i = m - 1; i >= 0; --i) {
      const T* row = Lc + (long)i * (i + 1) / 2;
      v[i] *= row[i];
      for (int j = 0; j < i; ++j) v[j] -= row[j] * v[i];
    }
  }
  const T u2 = f > T(0) ? d2 - A.two_l2 * log(f) : T(-1);
  const bool mean_live = u2 > T(0);
  const T u = mean_live ? sqrt(u2) : T(0);
  const T wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  T y[3] = {0, 0, 0};
  if (wn > T(0)) {
    const T gw = (gg[0] * w[0] + gg[1] * w[1] + gg[2] * w[2]) / wn;
    for (int d = 0; d < 3; ++d) y[d] = (gg[d] - gw * w[d] / wn) / wn;
  }
  const bool varf_live = VARF && (T(1) - vv) > T(0);
  const T m1 = M1 / S;
  const T h = zmin + m1;
  const T Vz = M2 / S - m1 * m1;
  // pass B: softmin coefficients c_i; V, P, d var / d alpha, sum c^2
  T V = 0, P = 0, dVa = 0, C2 = 0;
  for (int i = 0; i < m; ++i) {
    const T dx = l0 - p[4 * i], dy = l1 - p[4 * i + 1], dz = l2 - p[4 * i + 2];
    const T z = sqrt(dx * dx + dy * dy + dz * dz);
    const T si = exp(-A.alpha * (z - zmin)) / S;
    const T Bi = A.alpha * (h - z) + T(1);
    const T ci = si * Bi;
    V += sv[i] * ci * ci;
    P += sv[i] * ci * si;
    C2 += ci * ci;
    dVa += T(2) * sv[i] * ci * (si * (h - z) * (Bi + T(1)) - A.alpha * si * Vz);
  }
  // pass C: per-sample accumulations
  T dxv[3] = {0, 0, 0}, Hy[3] = {0, 0, 0}, Wz[3] = {0, 0, 0}, bk[3] = {0, 0, 0};
  T bkz = 0, bb = 0, El = 0, Es = 0, Eld[3] = {0, 0, 0}, Esd[3] = {0, 0, 0};
  for (int i = 0; i < m; ++i) {
    const T di[3] = {l0 - p[4 * i], l1 - p[4 * i + 1], l2 - p[4 * i + 2]};
    const T z2 = di[0] * di[0] + di[1] * di[1] + di[2] * di[2];
    const T z = sqrt(z2);
    const T e = exp(-(z2 - d2) * inv2l2);
    const T ae = p[4 * i + 3] * e;
    const T si = exp(-A.alpha * (z - zmin)) / S;
    const T ci = si * (A.alpha * (h - z) + T(1));
    const T dvdz = T(2) * A.alpha * (-sv[i] * ci * (ci + si) + si * V + ci * P);
    const T dy = di[0] * y[0] + di[1] * y[1] + di[2] * y[2];
    T kb = 0;
    if constexpr (VARF) kb = v[i] * e * ginv;
    for (int d = 0; d < 3; ++d) {
      if (z > T(0)) dxv[d] += dvdz * di[d] / z;
      Hy[d] += ae * dy * di[d];
      Wz[d] += ae * z2 * di[d];
      if constexpr (VARF) bk[d] += kb * di[d];
      Eld[d] += e * xi[XS * i] * di[d];
      Esd[d] += e * xi[XS * i + 1] * di[d];
    }
    if constexpr (VARF) {
      bkz += kb * z2;
      bb += v[i] * v[i];
    }
    El += e * xi[XS * i];
    Es += e * xi[XS * i + 1];
  }
  T bDb = 0;
  if (VARF && A.D && gf != T(0) && varf_live) {
    const T* Dc = A.D + A.loff[c];
    for (int i = 1; i < m; ++i) {
      const T* row = Dc + (long)i * (i + 1) / 2;
      T t = 0;
      for (int j = 0; j < i; ++j) t += row[j] * v[j];
      bDb += T(2) * v[i] * t;
    }
  }
  const T l3 = lt * lt * lt;
  // d_points
  for (int d = 0; d < 3; ++d) {
    T r = s * (f * y[d] - Hy[d] / (lt * lt)) + gv * dxv[d];
    if (mean_live) r += s * gm * w[d] / (f * u);
    if (varf_live) r += gf * T(2) * bk[d] / (lt * lt);
    out_dx[d] = r;
  }
  // weight cotangent . xi (through the fit)
  T aXl = s * (y[0] * Eld[0] + y[1] * Eld[1] + y[2] * Eld[2]);
  T aXs = s * (y[0] * Esd[0] + y[1] * Esd[1] + y[2] * Esd[2]);
  if (mean_live) {
    const T cm = -s * gm * lt * lt / (u * f);
    aXl += cm * El;
    aXs += cm * Es;
  }
  T dl = 0, ds = 0;
  if (mean_live) dl += s * gm * (u2 - Za / f) / (lt * u);
  dl += s * (y[0] * Wz[0] + y[1] * Wz[1] + y[2] * Wz[2]) / l3;
  if (A.alpha_tied) dl += gv * dVa * (-T(2) * A.alpha / lt);
  if (varf_live) dl += gf * (-T(2) * bkz / l3 + bDb);
  dl -= aXl;
  if (A.uniform_noise) {
    ds += gv * C2;
    if (varf_live) ds += gf * bb;
    ds -= aXs;
  }
  out_th[0] = (double)dl;
  out_th[1] = (double)ds;
}

// the per-query hyperparameter terms: FP64 models keep doubles; FP32 models keep
// float pairs (dl, ds), summed afterwards in float-float
template <class T>
__device__ __forceinline__ void store_theta(const BwdArgs<T>& A, long q, const double th[2]) {
  if constexpr (sizeof(T) == 8) {
    A.part[2 * q] = th[0];
    A.part[2 * q + 1] = th[1];
  } else {
    reinterpret_cast<float2*>(A.part)[q] = make_float2((float)th[0], (float)th[1]);
  }
}

template <class T, bool VARF>
__global__ void __launch_bounds__(BT) bwd_plain_kernel(BwdArgs<T> A) {
  const long q = (long)blockIdx.x * BT + threadIdx.x;
  if (q >= A.Q) return;
  int c = A.argmin[q];
  if (c >= A.n_cells) c = -1;   // not a cell of this model: no contribution
  T dx[3] = {T(0), T(0), T(0)};
  double th[2] = {0.0, 0.0};
  if (c < 0 && A.c_mean) {
    T gm, gv;
    mean_var_cotangents(A, q, gm, gv);   // the cost alone
  }
  if (c >= 0) {
    if constexpr (VARF) {
      T v[KSDF_MAX_M];
      query_vjp<T, true>(A, q, c, v, dx, th);
    } else {
      query_vjp<T, false>(A, q, c, nullptr, dx, th);
    }
  }
  for (int d = 0; d < 3; ++d) A.d_points[3 * q + d] = dx[d];
  store_theta(A, q, th);
}

// VJP of one query on its argmin cell for a Matern 3/2 model (Table I, App. D), in
// FP64 (FP64 models; vjp_matern_f32 below is the FP32 models' form).
// With c = sqrt(3)/l, the nearest sample distance d, e_i = exp(-c (z_i - d)),
// k'_i = (1 + c z_i) e_i, f' = sum a_i k'_i, w' = sum a_i e_i d_i (d_i = x - x_i):
//   u = d - ln(f')/c           du/dx = c w'/f',  du/dl|_a = (u - c Z/f')/l, Z = sum a e z^2,
//                              du/da_i = -k'_i / (c f')
//   g = w'/|w'|                dw'/dx = (sum a e) I - c sum a e d d^T / z,
//                              dw'/dc = -sum a e z d (dc/dl = -c/l),  dw'/da_i = e_i d_i
//   var_f = 1 - k^T A^{-1} k   d/dx = 2 c^2 sum beta_i e^{-c z_i} d_i,
//                              d/dl|_A = -2 c^2 sum beta_i z_i^2 e^{-c z_i} / l
// and the softmin variance as for the RBF.  The fit enters through the adjoint
// vectors xi_l = A^{-1} (dA/dl) a and xi_s = A^{-1} a as in query_vjp.
template <class T, bool VARF>
__device__ void vjp_matern(const BwdArgs<T>& A, long q, int c, double* v, double out_dx[3],
                           double out_th[2]) {
  constexpr bool F64 = sizeof(T) == 8;
  const double lt = F64 ? (double)A.ell : A.ell_d;
  const double al = F64 ? (double)A.alpha : A.alpha_d;
  const double mc = sqrt(3.0) / lt;
  const double x0 = A.pts[3 * q], x1 = A.pts[3 * q + 1], x2 = A.pts[3 * q + 2];
  const double s = A.sign ? (double)A.sign[q] : 1.0;
  T gmt, gvt;
  mean_var_cotangents(A, q, gmt, gvt);
  const double gm = gmt, gv = gvt;
  double gg[3] = {0, 0, 0};
  if (A.d_grad)
    for (int d = 0; d < 3; ++d) gg[d] = A.d_grad[3 * q + d];
  const double gf = VARF && A.d_var_f ? (double)A.d_var_f[q] : 0.0;
  const int b = A.offsets[c], m = A.offsets[c + 1] - b;
  const T* Lc = A.L + A.loff[c];
  const double l0 = x0 - A.centre64[3L * c], l1 = x1 - A.centre64[3L * c + 1],
               l2 = x2 - A.centre64[3L * c + 2];
  auto load = [&](int i, double di[3], double& pa) {
    if constexpr (F64) {
      const T* p = A.ps + 4L * (b + i);
      di[0] = l0 - p[0];
      di[1] = l1 - p[1];
      di[2] = l2 - p[2];
      pa = p[3];
    } else {
      const float* p = A.ps + 4L * (b + i);
      const float* pl = A.plo + 4L * (b + i);
      di[0] = l0 - ((double)p[0] + (double)pl[0]);
      di[1] = l1 - ((double)p[1] + (double)pl[1]);
      di[2] = l2 - ((double)p[2] + (double)pl[2]);
      pa = (double)p[3] + (double)pl[3];
    }
  };
  auto xi_l = [&](int i) -> double {
    if constexpr (F64) return A.xi[2L * (b + i)];
    else return (double)A.xi[4L * (b + i)] + (double)A.xi[4L * (b + i) + 2];
  };
  auto xi_s = [&](int i) -> double {
    if constexpr (F64) return A.xi[2L * (b + i) + 1];
    else return (double)A.xi[4L * (b + i) + 1] + (double)A.xi[4L * (b + i) + 3];
  };
  double d2 = INFINITY;
  for (int i = 0; i < m; ++i) {
    double di[3], pa;
    load(i, di, pa);
    d2 = fmin(d2, di[0] * di[0] + di[1] * di[1] + di[2] * di[2]);
  }
  const double zmin = sqrt(d2);
  // pass A: f', sum a e, w', Z, softmin moments, k
  double f = 0, fe = 0, w[3] = {0, 0, 0}, Za = 0, S = 0, M1 = 0, M2 = 0;
  for (int i = 0; i < m; ++i) {
    double di[3], pa;
    load(i, di, pa);
    const double z2 = di[0] * di[0] + di[1] * di[1] + di[2] * di[2];
    const double z = sqrt(z2);
    const double e = exp(-mc * (z - zmin));
    f += pa * (1.0 + mc * z) * e;
    fe += pa * e;
    for (int d = 0; d < 3; ++d) w[d] += pa * e * di[d];
    Za += pa * e * z2;
    const double t = z - zmin;
    const double sm = exp(-al * t);
    S += sm;
    M1 += sm * t;
    M2 += sm * t * t;
    if constexpr (VARF) v[i] = (1.0 + mc * z) * exp(-mc * z);
  }
  double vv = 0;
  if constexpr (VARF) {
    for (int i = 0; i < m; ++i) {
      const T* row = Lc + (long)i * (i + 1) / 2;
      double t = v[i];
      for (int j = 0; j < i; ++j) t -= (double)row[j] * v[j];
      v[i] = t * (double)row[i];
      vv += v[i] * v[i];
    }
    for (int i = m - 1; i >= 0; --i) {
      const T* row = Lc + (long)i * (i + 1) / 2;
      v[i] *= (double)row[i];
      for (int j = 0; j < i; ++j) v[j] -= (double)row[j] * v[i];
    }
  }
  const double u = f > 0.0 ? zmin - log(f) / mc : -1.0;
  const bool mean_live = u > 0.0;
  const double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  double y[3] = {0, 0, 0};
  if (wn > 0.0) {
    const double gw = (gg[0] * w[0] + gg[1] * w[1] + gg[2] * w[2]) / wn;
    for (int d = 0; d < 3; ++d) y[d] = (gg[d] - gw * w[d] / wn) / wn;
  }
  const bool varf_live = VARF && (1.0 - vv) > 0.0;
  const double m1 = M1 / S;
  const double h = zmin + m1;
  const double Vz = M2 / S - m1 * m1;
  double V = 0, P = 0, dVa = 0, C2 = 0;
  for (int i = 0; i < m; ++i) {
    double di[3], pa;
    load(i, di, pa);
    const double z = sqrt(di[0] * di[0] + di[1] * di[1] + di[2] * di[2]);
    const double si = exp(-al * (z - zmin)) / S;
    const double Bi = al * (h - z) + 1.0;
    const double ci = si * Bi;
    const double svi = A.sv[b + i];
    V += svi * ci * ci;
    P += svi * ci * si;
    C2 += ci * ci;
    dVa += 2.0 * svi * ci * (si * (h - z) * (Bi + 1.0) - al * si * Vz);
  }
  double dxv[3] = {0, 0, 0}, Hy[3] = {0, 0, 0}, Wz[3] = {0, 0, 0}, bk[3] = {0, 0, 0};
  double bkz = 0, bb = 0, El = 0, Es = 0, Eld[3] = {0, 0, 0}, Esd[3] = {0, 0, 0};
  for (int i = 0; i < m; ++i) {
    double di[3], pa;
    load(i, di, pa);
    const double z2 = di[0] * di[0] + di[1] * di[1] + di[2] * di[2];
    const double z = sqrt(z2);
    const double e = exp(-mc * (z - zmin));
    const double kp = (1.0 + mc * z) * e;
    const double ae = pa * e;
    const double si = exp(-al * (z - zmin)) / S;
    const double ci = si * (al * (h - z) + 1.0);
    const double svi = A.sv[b + i];
    const double dvdz = 2.0 * al * (-svi * ci * (ci + si) + si * V + ci * P);
    const double dy = di[0] * y[0] + di[1] * y[1] + di[2] * y[2];
    double kb = 0;
    if constexpr (VARF) kb = v[i] * exp(-mc * z);
    const double xl = xi_l(i), xs = xi_s(i);
    for (int d = 0; d < 3; ++d) {
      if (z > 0.0) {
        dxv[d] += dvdz * di[d] / z;
        Hy[d] += ae * dy * di[d] / z;
      }
      Wz[d] += ae * z * di[d];
      if constexpr (VARF) bk[d] += kb * di[d];
      Eld[d] += e * xl * di[d];
      Esd[d] += e * xs * di[d];
    }
    if constexpr (VARF) {
      bkz += kb * z2;
      bb += v[i] * v[i];
    }
    El += kp * xl;
    Es += kp * xs;
  }
  double bDb = 0;
  if (VARF && A.D && gf != 0.0 && varf_live) {
    const T* Dc = A.D + A.loff[c];
    for (int i = 1; i < m; ++i) {
      const T* row = Dc + (long)i * (i + 1) / 2;
      double t = 0;
      for (int j = 0; j < i; ++j) t += (double)row[j] * v[j];
      bDb += 2.0 * v[i] * t;
    }
  }
  for (int d = 0; d < 3; ++d) {
    double r = s * (fe * y[d] - mc * Hy[d]) + gv * dxv[d];
    if (mean_live) r += s * gm * mc * w[d] / f;
    if (varf_live) r += gf * 2.0 * mc * mc * bk[d];
    out_dx[d] = r;
  }
  double aXl = s * (y[0] * Eld[0] + y[1] * Eld[1] + y[2] * Eld[2]);
  double aXs = s * (y[0] * Esd[0] + y[1] * Esd[1] + y[2] * Esd[2]);
  if (mean_live) {
    const double cm = -s * gm / (mc * f);
    aXl += cm * El;
    aXs += cm * Es;
  }
  double dl = 0, ds = 0;
  if (mean_live) dl += s * gm * (u - mc * Za / f) / lt;
  dl += s * (mc / lt) * (y[0] * Wz[0] + y[1] * Wz[1] + y[2] * Wz[2]);
  if (A.alpha_tied) dl += gv * dVa * (-2.0 * al / lt);
  if (varf_live) dl += gf * (-2.0 * mc * mc * bkz / lt + bDb);
  dl -= aXl;
  if (A.uniform_noise) {
    ds += gv * C2;
    if (varf_live) ds += gf * bb;
    ds -= aXs;
  }
  out_th[0] = dl;
  out_th[1] = ds;
}

// Compensated FP32 sum (TwoSum, Knuth): the running sum and the sum of its rounding
// errors, so that m terms carry about one rounding of the result instead of m.
struct CAcc {
  float s = 0.f, c = 0.f;
  __device__ __forceinline__ void add(float x) {
#pragma clang fp contract(off)
    const float t = s + x;
    const float bb = t - s;
    c += (s - (t - bb)) + (x - bb);
    s = t;
  }
  __device__ __forceinline__ float val() const { return s + c; }
};

// The Matern 3/2 VJP of one query for an FP32 model, in FP32: the same sums as
// vjp_matern, with the differences to the samples exact as float pairs, z_i and
// z_i - d as float pairs (the square root by one Newton step), the exponentials from
// float-pair arguments (the hardware 2^x on the fraction, the low part to first
// order), and the sums whose terms cancel accumulated with compensation.  With VARF
// the triangular solves for A^{-1} k run in FP32 on the factor (as query_vjp).
template <bool VARF>
__device__ void vjp_matern_f32(const BwdArgs<float>& A, long q, int c, float* v, float out_dx[3],
                               double out_th[2]) {
  const float lt = A.ell, al = A.alpha;
  const float mc = A.mc_ff[0];
  const ff mclf{A.mcl_ff[0], A.mcl_ff[1]};
  const float x0 = A.pts[3 * q], x1 = A.pts[3 * q + 1], x2 = A.pts[3 * q + 2];
  const float s = A.sign ? (float)A.sign[q] : 1.f;
  float gm, gv;
  mean_var_cotangents(A, q, gm, gv);
  float gg[3] = {0.f, 0.f, 0.f};
  if (A.d_grad)
    for (int d = 0; d < 3; ++d) gg[d] = A.d_grad[3 * q + d];
  const float gf = VARF && A.d_var_f ? A.d_var_f[q] : 0.f;
  const int b = A.offsets[c], m = A.offsets[c + 1] - b;
  const float* Lc = A.L + A.loff[c];
  const float4* P4 = reinterpret_cast<const float4*>(A.ps);
  const float4* PL = reinterpret_cast<const float4*>(A.plo);
  const float4* X4 = reinterpret_cast<const float4*>(A.xi);
  const ff lx = ff_two_sum(x0, -(float)A.centre64[3L * c]);
  const ff ly = ff_two_sum(x1, -(float)A.centre64[3L * c + 1]);
  const ff lz = ff_two_sum(x2, -(float)A.centre64[3L * c + 2]);
  auto load = [&](int i, float di[3], ff& z2, float& pa) {
    const float4 h = P4[b + i], lo = PL[b + i];
    const ff dx = ff_sub_lean(lx.hi, lx.lo, h.x, lo.x);
    const ff dy = ff_sub_lean(ly.hi, ly.lo, h.y, lo.y);
    const ff dz = ff_sub_lean(lz.hi, lz.lo, h.z, lo.z);
    di[0] = dx.hi;
    di[1] = dy.hi;
    di[2] = dz.hi;
    z2 = ff_norm2_lean(dx, dy, dz);
    pa = h.w + lo.w;
  };
  // e^{-c t} for a float-pair t >= 0 as 2^{-c log2(e) t}
  auto expc = [&](ff t) {
    const ff u = ff_mul(t, mclf);
    const float n = floorf(u.hi);
    const float e = __builtin_amdgcn_exp2f(n - u.hi) * (1.f - 0.6931471805599453f * u.lo);
    return ldexpf(e, -(int)n);
  };
  ff d2f{INFINITY, 0.f};
  for (int i = 0; i < m; ++i) {
    float di[3], pa;
    ff z2;
    load(i, di, z2, pa);
    if (z2.hi < d2f.hi || (z2.hi == d2f.hi && z2.lo < d2f.lo)) d2f = z2;
  }
  const ff zminf = ff_sqrt(d2f);
  const float zmin = zminf.hi + zminf.lo;
  // pass A: f', sum a e, w', Z, softmin moments, k
  CAcc f, fe, w[3], Za;
  float S = 0.f, M1 = 0.f, M2 = 0.f;
  for (int i = 0; i < m; ++i) {
    float di[3], pa;
    ff z2f;
    load(i, di, z2f, pa);
    const ff zf = ff_sqrt(z2f);
    const float z = zf.hi + zf.lo, z2 = z2f.hi + z2f.lo;
    const ff tf = ff_sub_lean(zf.hi, zf.lo, zminf.hi, zminf.lo);
    const float e = expc(tf);
    const float ae = pa * e;
    f.add(ae * fmaf(mc, z, 1.f));
    fe.add(ae);
    w[0].add(ae * di[0]);
    w[1].add(ae * di[1]);
    w[2].add(ae * di[2]);
    Za.add(ae * z2);
    const float t = tf.hi + tf.lo;
    const float sm = __builtin_amdgcn_exp2f(-1.4426950408889634f * al * t);
    S += sm;
    M1 += sm * t;
    M2 += sm * t * t;
    if constexpr (VARF) v[i] = fmaf(mc, z, 1.f) * expc(zf);
  }
  float vv = 0.f;
  if constexpr (VARF) {
    for (int i = 0; i < m; ++i) {
      const float* row = Lc + (long)i * (i + 1) / 2;
      float t = v[i];
      for (int j = 0; j < i; ++j) t -= row[j] * v[j];
      v[i] = t * row[i];
      vv += v[i] * v[i];
    }
    for (int i = m - 1; i >= 0; --i) {
      const float* row = Lc + (long)i * (i + 1) / 2;
      v[i] *= row[i];
      for (int j = 0; j < i; ++j) v[j] -= row[j] * v[i];
    }
  }
  const float fv = f.val(), fev = fe.val();
  const float wv[3] = {w[0].val(), w[1].val(), w[2].val()};
  const float u = fv > 0.f ? zmin - logf(fv) / mc : -1.f;
  const bool mean_live = u > 0.f;
  const float wn = sqrtf(wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2]);
  float y[3] = {0.f, 0.f, 0.f};
  if (wn > 0.f) {
    const float gw = (gg[0] * wv[0] + gg[1] * wv[1] + gg[2] * wv[2]) / wn;
    for (int d = 0; d < 3; ++d) y[d] = (gg[d] - gw * wv[d] / wn) / wn;
  }
  const bool varf_live = VARF && (1.f - vv) > 0.f;
  const float iS = 1.f / S;
  const float m1 = M1 * iS;
  const float h = zmin + m1;
  const float Vz = M2 * iS - m1 * m1;
  float V = 0.f, Pp = 0.f, dVa = 0.f, C2 = 0.f;
  for (int i = 0; i < m; ++i) {
    float di[3], pa;
    ff z2f;
    load(i, di, z2f, pa);
    const ff zf = ff_sqrt(z2f);
    const ff tf = ff_sub_lean(zf.hi, zf.lo, zminf.hi, zminf.lo);
    const float z = zf.hi + zf.lo, t = tf.hi + tf.lo;
    const float si = __builtin_amdgcn_exp2f(-1.4426950408889634f * al * t) * iS;
    const float Bi = al * (h - z) + 1.f;
    const float ci = si * Bi;
    const float svi = A.sv[b + i];
    V += svi * ci * ci;
    Pp += svi * ci * si;
    C2 += ci * ci;
    dVa += 2.f * svi * ci * (si * (h - z) * (Bi + 1.f) - al * si * Vz);
  }
  float dxv[3] = {0.f, 0.f, 0.f}, bk[3] = {0.f, 0.f, 0.f};
  CAcc Hy[3], Wz[3], El, Es, Eld[3], Esd[3];
  float bkz = 0.f, bb = 0.f;
  for (int i = 0; i < m; ++i) {
    float di[3], pa;
    ff z2f;
    load(i, di, z2f, pa);
    const ff zf = ff_sqrt(z2f);
    const ff tf = ff_sub_lean(zf.hi, zf.lo, zminf.hi, zminf.lo);
    const float z = zf.hi + zf.lo, z2 = z2f.hi + z2f.lo, t = tf.hi + tf.lo;
    const float e = expc(tf);
    const float kp = fmaf(mc, z, 1.f) * e;
    const float ae = pa * e;
    const float si = __builtin_amdgcn_exp2f(-1.4426950408889634f * al * t) * iS;
    const float ci = si * (al * (h - z) + 1.f);
    const float svi = A.sv[b + i];
    const float dvdz = 2.f * al * (-svi * ci * (ci + si) + si * V + ci * Pp);
    const float dy = di[0] * y[0] + di[1] * y[1] + di[2] * y[2];
    float kb = 0.f;
    if constexpr (VARF) kb = v[i] * expc(zf);
    const float4 xq = X4[b + i];
    const float xl = xq.x + xq.z, xs = xq.y + xq.w;
    const float rz = z > 0.f ? 1.f / z : 0.f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      dxv[d] += dvdz * di[d] * rz;
      Hy[d].add(ae * dy * di[d] * rz);
      Wz[d].add(ae * z * di[d]);
      if constexpr (VARF) bk[d] += kb * di[d];
      Eld[d].add(e * xl * di[d]);
      Esd[d].add(e * xs * di[d]);
    }
    if constexpr (VARF) {
      bkz += kb * z2;
      bb += v[i] * v[i];
    }
    El.add(kp * xl);
    Es.add(kp * xs);
  }
  float bDb = 0.f;
  if (VARF && A.D && gf != 0.f && varf_live) {
    const float* Dc = A.D + A.loff[c];
    for (int i = 1; i < m; ++i) {
      const float* row = Dc + (long)i * (i + 1) / 2;
      float t = 0.f;
      for (int j = 0; j < i; ++j) t += row[j] * v[j];
      bDb += 2.f * v[i] * t;
    }
  }
  for (int d = 0; d < 3; ++d) {
    float r = s * (fev * y[d] - mc * Hy[d].val()) + gv * dxv[d];
    if (mean_live) r += s * gm * mc * wv[d] / fv;
    if (varf_live) r += gf * 2.f * mc * mc * bk[d];
    out_dx[d] = r;
  }
  float aXl = s * (y[0] * Eld[0].val() + y[1] * Eld[1].val() + y[2] * Eld[2].val());
  float aXs = s * (y[0] * Esd[0].val() + y[1] * Esd[1].val() + y[2] * Esd[2].val());
  if (mean_live) {
    const float cm = -s * gm / (mc * fv);
    aXl += cm * El.val();
    aXs += cm * Es.val();
  }
  float dl = 0.f, ds = 0.f;
  if (mean_live) dl += s * gm * (u - mc * Za.val() / fv) / lt;
  dl += s * (mc / lt) * (y[0] * Wz[0].val() + y[1] * Wz[1].val() + y[2] * Wz[2].val());
  if (A.alpha_tied) dl += gv * dVa * (-2.f * al / lt);
  if (varf_live) dl += gf * (-2.f * mc * mc * bkz / lt + bDb);
  dl -= aXl;
  if (A.uniform_noise) {
    ds += gv * C2;
    if (varf_live) ds += gf * bb;
    ds -= aXs;
  }
  out_th[0] = (double)dl;
  out_th[1] = (double)ds;
}

template <class T, bool VARF>
__global__ void __launch_bounds__(BT) bwd_matern_kernel(BwdArgs<T> A) {
  const long q = (long)blockIdx.x * BT + threadIdx.x;
  if (q >= A.Q) return;
  int c = A.argmin[q];
  if (c >= A.n_cells) c = -1;
  double dx[3] = {0, 0, 0}, th[2] = {0, 0};
  if (c < 0 && A.c_mean) {
    T gm, gv;
    mean_var_cotangents(A, q, gm, gv);   // the cost alone
  }
  if (c >= 0) {
    if constexpr (sizeof(T) == 4) {
      float fdx[3];
      if constexpr (VARF) {
        float v[KSDF_MAX_M];
        vjp_matern_f32<true>(A, q, c, v, fdx, th);
      } else {
        vjp_matern_f32<false>(A, q, c, nullptr, fdx, th);
      }
      for (int d = 0; d < 3; ++d) dx[d] = fdx[d];
    } else if constexpr (VARF) {
      double v[KSDF_MAX_M];
      vjp_matern<T, true>(A, q, c, v, dx, th);
    } else {
      vjp_matern<T, false>(A, q, c, nullptr, dx, th);
    }
  }
  for (int d = 0; d < 3; ++d) A.d_points[3 * q + d] = (T)dx[d];
  store_theta(A, q, th);
}


// VJP of one query on its argmin cell for an FP32 model, in FP32.  Each term carries
// about one float rounding (cell-local differences from the float-float store, the
// kernel value from the hardware 2^x), and the sums whose terms cancel -- f' = sum
// a_i e_i, w', Z, the kernel-Hessian and z^2-weighted vectors and the fit's adjoint
// sums sum e_i xi_i -- are accumulated with compensation, so that their error is a
// few roundings of the terms rather than of the sum; the softmin sums (positive
// terms) are plain.  The per-query hyperparameter terms leave in FP64 for the
// fixed-order reduction.  UNI: the cell is wave-uniform (scalar loads).
constexpr int BCH = 2;

template <bool UNI>
__device__ __forceinline__ void vjp_f32(const BwdArgs<float>& A, float x0, float x1, float x2,
                                        float s, float gm, const float gg[3], float gv, int c,
                                        float out_dx[3], double out_th[2]) {
  const float4* __restrict__ P4 = reinterpret_cast<const float4*>(A.ps);
  const float4* __restrict__ PL = reinterpret_cast<const float4*>(A.plo);
  const float4* __restrict__ X4 = reinterpret_cast<const float4*>(A.xi);
  const float* __restrict__ SV = A.sv;
  const int b = UNI ? __builtin_amdgcn_readfirstlane(A.offsets[c]) : A.offsets[c];
  const int m = (UNI ? __builtin_amdgcn_readfirstlane(A.offsets[c + 1]) : A.offsets[c + 1]) - b;
  const float lt = A.ell, two_l2 = A.two_l2, al = A.alpha;
  const float ca = 1.4426950408889634f * al;
  // the query in the cell's frame, exact as a float pair (the store's coordinates are
  // relative to the float centre)
  const ff lx = ff_two_sum(x0, -(float)A.centre64[3L * c]);
  const ff ly = ff_two_sum(x1, -(float)A.centre64[3L * c + 1]);
  const ff lz = ff_two_sum(x2, -(float)A.centre64[3L * c + 2]);
  // the differences to sample i (float), and |x - x_i|^2 as a float-float pair from
  // the exact differences, so that the kernel exponent keeps its precision where it
  // is large (far samples of big cells)
  auto diff = [&](int i, float di[3], ff& z2) {
    const float4 h = P4[b + i], lo = PL[b + i];
    const ff dx = ff_sub_lean(lx.hi, lx.lo, h.x, lo.x);
    const ff dy = ff_sub_lean(ly.hi, ly.lo, h.y, lo.y);
    const ff dz = ff_sub_lean(lz.hi, lz.lo, h.z, lo.z);
    di[0] = dx.hi;
    di[1] = dy.hi;
    di[2] = dz.hi;
    z2 = ff_norm2_lean(dx, dy, dz);
  };
  // e = exp(-(z2 - d2) / (2 l^2)) = 2^-t with t = (z2 - d2) log2(e) / (2 l^2) formed
  // in float-float: the hardware 2^x on the fraction of t.hi, the low part by its
  // first-order term
  const ff c2f{A.c2_ff[0], A.c2_ff[1]};
  auto kval = [&](ff z2, ff d2f) {
    const ff t = ff_mul(ff_sub_lean(z2.hi, z2.lo, d2f.hi, d2f.lo), c2f);
    const float n = floorf(t.hi);
    const float e = __builtin_amdgcn_exp2f(n - t.hi) * (1.f - 0.6931471805599453f * t.lo);
    return ldexpf(e, -(int)n);
  };
  auto weight = [&](int i) {
    const float4 h = P4[b + i], lo = PL[b + i];
    return h.w + lo.w;
  };
  ff d2f{INFINITY, 0.f};
  for (int i0 = 0; i0 < m; i0 += BCH) {
#pragma unroll
    for (int j = 0; j < BCH; ++j) {
      float di[3];
      ff z2;
      diff(i0 + j, di, z2);   // the store is padded
      if (i0 + j < m && (z2.hi < d2f.hi || (z2.hi == d2f.hi && z2.lo < d2f.lo))) d2f = z2;
    }
  }
  const float d2 = d2f.hi + d2f.lo;
  const float zmin = sqrtf(d2);
  // pass A: f', w', Z, softmin moments
  CAcc f, w[3], Za;
  float S = 0.f, M1 = 0.f, M2 = 0.f;
  for (int i0 = 0; i0 < m; i0 += BCH) {
#pragma unroll
    for (int j = 0; j < BCH; ++j) {
      const bool ok = i0 + j < m;
      float di[3];
      ff z2f;
      diff(i0 + j, di, z2f);
      const float z2 = z2f.hi + z2f.lo;
      const float e = ok ? kval(z2f, d2f) : 0.f;
      const float ae = weight(i0 + j) * e;
      f.add(ae);
      w[0].add(ae * di[0]);
      w[1].add(ae * di[1]);
      w[2].add(ae * di[2]);
      Za.add(ae * z2);
      const float t = sqrtf(z2) - zmin;
      const float sm = ok ? __builtin_amdgcn_exp2f(-ca * t) : 0.f;
      S += sm;
      M1 += sm * t;
      M2 += sm * t * t;
    }
  }
  const float fv = f.val();
  const float wv[3] = {w[0].val(), w[1].val(), w[2].val()};
  const float u2 = fv > 0.f ? d2 - two_l2 * logf(fv) : -1.f;
  const bool mean_live = u2 > 0.f;
  const float u = mean_live ? sqrtf(u2) : 0.f;
  const float wn = sqrtf(wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2]);
  float y[3] = {0.f, 0.f, 0.f};
  if (wn > 0.f) {
    const float gw = (gg[0] * wv[0] + gg[1] * wv[1] + gg[2] * wv[2]) / wn;
    for (int d = 0; d < 3; ++d) y[d] = (gg[d] - gw * wv[d] / wn) / wn;
  }
  const float iS = 1.f / S;
  const float m1 = M1 * iS;
  const float h = zmin + m1;
  const float Vz = M2 * iS - m1 * m1;
  // pass B: every per-sample sum at once.  d var / d z_j = 2 alpha (-sigma_j^2 c_j
  // (c_j + s_j) + s_j V + c_j P) needs V and P of the same pass, so the point
  // derivative keeps its three parts apart (Q1, Q2, Q3) and combines them after.
  float V = 0.f, Pp = 0.f, dVa = 0.f, C2 = 0.f;
  float Q1[3] = {0.f, 0.f, 0.f}, Q2[3] = {0.f, 0.f, 0.f}, Q3[3] = {0.f, 0.f, 0.f};
  CAcc Hy[3], Wz[3], El, Es, Eld[3], Esd[3];
  for (int i0 = 0; i0 < m; i0 += BCH) {
#pragma unroll
    for (int j = 0; j < BCH; ++j) {
      const bool ok = i0 + j < m;
      float di[3];
      ff z2f;
      diff(i0 + j, di, z2f);
      const float4 xq = X4[b + i0 + j];
      const float svj = ok ? SV[b + i0 + j] : 0.f;
      const float x0j = ok ? xq.x + xq.z : 0.f;
      const float x1j = ok ? xq.y + xq.w : 0.f;
      const float z2 = z2f.hi + z2f.lo;
      const float z = sqrtf(z2);
      const float e = ok ? kval(z2f, d2f) : 0.f;
      const float ae = weight(i0 + j) * e;
      const float si = ok ? __builtin_amdgcn_exp2f(-ca * (z - zmin)) * iS : 0.f;
      const float Bi = al * (h - z) + 1.f;
      const float ci = si * Bi;
      V += svj * ci * ci;
      Pp += svj * ci * si;
      C2 += ci * ci;
      dVa += 2.f * svj * ci * (si * (h - z) * (Bi + 1.f) - al * si * Vz);
      const float rz = z > 0.f ? 1.f / z : 0.f;
      const float q1 = -svj * ci * (ci + si) * rz, q2 = si * rz, q3 = ci * rz;
      const float dy = di[0] * y[0] + di[1] * y[1] + di[2] * y[2];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        Q1[d] += q1 * di[d];
        Q2[d] += q2 * di[d];
        Q3[d] += q3 * di[d];
        Hy[d].add(ae * dy * di[d]);
        Wz[d].add(ae * z2 * di[d]);
        Eld[d].add(e * x0j * di[d]);
        Esd[d].add(e * x1j * di[d]);
      }
      El.add(e * x0j);
      Es.add(e * x1j);
    }
  }
  const float l3 = lt * lt * lt;
  for (int d = 0; d < 3; ++d) {
    const float dxv = 2.f * al * (Q1[d] + V * Q2[d] + Pp * Q3[d]);
    float r = s * (fv * y[d] - Hy[d].val() / (lt * lt)) + gv * dxv;
    if (mean_live) r += s * gm * wv[d] / (fv * u);
    out_dx[d] = r;
  }
  float aXl = s * (y[0] * Eld[0].val() + y[1] * Eld[1].val() + y[2] * Eld[2].val());
  float aXs = s * (y[0] * Esd[0].val() + y[1] * Esd[1].val() + y[2] * Esd[2].val());
  if (mean_live) {
    const float cm = -s * gm * lt * lt / (u * fv);
    aXl += cm * El.val();
    aXs += cm * Es.val();
  }
  float dl = 0.f, ds = 0.f;
  if (mean_live) dl += s * gm * (u2 - Za.val() / fv) / (lt * u);
  dl += s * (y[0] * Wz[0].val() + y[1] * Wz[1].val() + y[2] * Wz[2].val()) / l3;
  if (A.alpha_tied) dl += gv * dVa * (-2.f * al / lt);
  dl -= aXl;
  if (A.uniform_noise) ds += gv * C2 - aXs;
  out_th[0] = (double)dl;
  out_th[1] = (double)ds;
}

// FP32: lanes take queries in argmin-cell order (perm), and each wave walks the
// distinct argmin cells of its lanes -- after the sort usually one or two -- so the
// cell index is wave-uniform and the cell's samples, factor and adjoint vectors are
// read through scalar loads.
template <bool VARF, bool LANE>
__global__ void __launch_bounds__(BT) bwd_wave_kernel(BwdArgs<float> A, const int* perm) {
  const long sq = (long)blockIdx.x * BT + threadIdx.x;
  const bool active = sq < A.Q;
  const long q = active ? perm[sq] : 0;
  int bc = active ? A.argmin[q] : -1;
  if (bc >= A.n_cells) bc = -1;
  float dx[3] = {0.f, 0.f, 0.f};
  double th[2] = {0.0, 0.0};
  bool todo = bc >= 0;
  // per-lane inputs (the no-var_f path reads them once for all its cells)
  const float x0 = A.pts[3 * q], x1 = A.pts[3 * q + 1], x2 = A.pts[3 * q + 2];
  const float sgn = A.sign ? (float)A.sign[q] : 1.f;
  float gm = 0.f, gv = 0.f;
  if (active) mean_var_cotangents(A, q, gm, gv);
  float gg[3] = {0.f, 0.f, 0.f};
  if (A.d_grad)
    for (int d = 0; d < 3; ++d) gg[d] = A.d_grad[3 * q + d];
  if constexpr (LANE && !VARF) {
    // per lane (sparse queries): every lane its own argmin cell, in one round
    if (__ballot(todo)) {
      float tdx[3];
      double tth[2];
      vjp_f32<false>(A, x0, x1, x2, sgn, gm, gg, gv, todo ? bc : 0, tdx, tth);
      if (todo) {
        for (int d = 0; d < 3; ++d) dx[d] = tdx[d];
        th[0] = tth[0];
        th[1] = tth[1];
        todo = false;
      }
    }
  }
  while (true) {
    unsigned key = todo ? (unsigned)bc : 0xffffffffu;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) key = min(key, (unsigned)__shfl_xor((int)key, o, 64));
    key = (unsigned)__builtin_amdgcn_readfirstlane((int)key);
    if (key == 0xffffffffu) break;
    const int c = (int)key;
    if constexpr (VARF) {
      if (todo && bc == c) {
        float v[KSDF_MAX_M];
        query_vjp<float, true>(A, q, c, v, dx, th);
        todo = false;
      }
    } else {
      float tdx[3];
      double tth[2];
      vjp_f32<true>(A, x0, x1, x2, sgn, gm, gg, gv, c, tdx, tth);
      if (todo && bc == c) {
        for (int d = 0; d < 3; ++d) dx[d] = tdx[d];
        th[0] = tth[0];
        th[1] = tth[1];
        todo = false;
      }
    }
  }
  if (!active) return;
  for (int d = 0; d < 3; ++d) A.d_points[3 * q + d] = dx[d];
  store_theta(A, q, th);
}

// Counting sort of the queries by argmin cell (queries without a cell go last).
constexpr int ST = 256;
__global__ void fill_int_kernel(int* p, long n, int v) {
  const long i = (long)blockIdx.x * ST + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void __launch_bounds__(ST) argmin_count_kernel(const int* argmin, long Q, int n_cells,
                                                          int* key, int* count) {
  const long q = (long)blockIdx.x * ST + threadIdx.x;
  const bool valid = q < Q;
  int c = valid ? argmin[q] : n_cells;
  if (c < 0 || c >= n_cells) c = n_cells;
  if (valid) key[q] = c;
  wave_count(count, c, valid);   // consecutive queries mostly share their cell
}
// exclusive scan of count[0..n) into start (one block; n is a cell count)
__global__ void __launch_bounds__(1024) scan_counts_kernel(const int* count, int n, int* start) {
  __shared__ int part[1024];
  const int per = (n + 1023) / 1024;
  const int beg = threadIdx.x * per;
  const int end = beg + per < n ? beg + per : n;
  int t = 0;
  for (int i = beg; i < end; ++i) t += count[i];
  part[threadIdx.x] = t;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int add = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  int run = threadIdx.x ? part[threadIdx.x - 1] : 0;
  for (int i = beg; i < end; ++i) {
    start[i] = run;
    run += count[i];
  }
}
__global__ void __launch_bounds__(ST) argmin_scatter_kernel(long Q, const int* key, int* cursor,
                                                            int* perm) {
  const long q = (long)blockIdx.x * ST + threadIdx.x;
  const bool valid = q < Q;
  const int pos = wave_slot(cursor, valid ? key[q] : 0, valid);
  if (valid) perm[pos] = (int)q;
}

// Deterministic FP64 reduction of the per-query hyperparameter partials: RB blocks each
// sum a fixed contiguous chunk (coalesced, fixed tree), then one block sums the RB
// partials in a fixed tree.  The order depends on Q only.
constexpr int RT = 256;
constexpr int RB = 256;
__device__ void block_sum2(double a, double b, double* out) {
  __shared__ double r0[RT], r1[RT];
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = b;
  __syncthreads();
  for (int o = RT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      r0[threadIdx.x] += r0[threadIdx.x + o];
      r1[threadIdx.x] += r1[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = r0[0];
    out[1] = r1[0];
  }
}
__global__ void __launch_bounds__(RT) theta_partial_kernel(const double* part, long Q, double* red) {
  const long per = (Q + RB - 1) / RB;
  const long beg = (long)blockIdx.x * per;
  const long end = beg + per < Q ? beg + per : Q;
  double a = 0.0, b = 0.0;
  for (long i = beg + threadIdx.x; i < end; i += RT) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  block_sum2(a, b, red + 2 * blockIdx.x);
}
__global__ void __launch_bounds__(RT) theta_final_kernel(const double* red, double* out) {
  block_sum2(red[2 * threadIdx.x], red[2 * threadIdx.x + 1], out);
}

// The same fixed-order reduction for FP32 models, in float-float: the per-query float
// pairs, RB block partials (hi, lo) x 2, then one block; the result leaves as the
// double hi + lo.
__device__ void block_sum2_ff(ff a, ff b, float4* out) {
  __shared__ float r0h[RT], r0l[RT], r1h[RT], r1l[RT];
  r0h[threadIdx.x] = a.hi;
  r0l[threadIdx.x] = a.lo;
  r1h[threadIdx.x] = b.hi;
  r1l[threadIdx.x] = b.lo;
  __syncthreads();
  for (int o = RT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const int t = threadIdx.x;
      const ff x = ff_add(ff{r0h[t], r0l[t]}, ff{r0h[t + o], r0l[t + o]});
      const ff y = ff_add(ff{r1h[t], r1l[t]}, ff{r1h[t + o], r1l[t + o]});
      r0h[t] = x.hi;
      r0l[t] = x.lo;
      r1h[t] = y.hi;
      r1l[t] = y.lo;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = make_float4(r0h[0], r0l[0], r1h[0], r1l[0]);
}
__global__ void __launch_bounds__(RT) theta_partial32_kernel(const float2* part, long Q, float4* red) {
  const long per = (Q + RB - 1) / RB;
  const long beg = (long)blockIdx.x * per;
  const long end = beg + per < Q ? beg + per : Q;
  ff a{0.f, 0.f}, b{0.f, 0.f};
  for (long i = beg + threadIdx.x; i < end; i += RT) {
    const float2 v = part[i];
    a = ff_add(a, ff{v.x, 0.f});
    b = ff_add(b, ff{v.y, 0.f});
  }
  block_sum2_ff(a, b, red + blockIdx.x);
}
__global__ void __launch_bounds__(RT) theta_final32_kernel(const float4* red, double* out) {
  const float4 v = red[threadIdx.x];
  __shared__ float4 r;
  block_sum2_ff(ff{v.x, v.y}, ff{v.z, v.w}, &r);
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = (double)r.x + (double)r.y;
    out[1] = (double)r.z + (double)r.w;
  }
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t backward_workspace_bytes(const ksdf_model* m, long Q) {
  const size_t fb = m->precision == KSDF_FP64 ? sizeof(double) : sizeof(float);
  const size_t nc = (size_t)m->n_cells + 1;
  // per-query theta partials, block partials, the argmin sort (key, perm, count,
  // cursor), and (when no argmin is passed) a forward pass
  return al256(2 * Q * sizeof(double)) + al256(2 * RB * sizeof(double)) +
         2 * al256(Q * sizeof(int)) + 2 * al256(nc * sizeof(int)) + al256(Q * sizeof(int)) +
         al256(Q * 5 * fb) + al256(query_workspace_bytes(m, Q));
}

int launch_backward(const ksdf_model* m, const void* points, long Q, const int8_t* sign,
                    const int* argmin, const void* d_mean, const void* d_grad, const void* d_var,
                    const void* d_var_f, void* d_points, double* d_hyper, void* ws,
                    size_t ws_bytes, hipStream_t s, const CostArgs* cost) {
  if (!m->adjoint) {
    set_error("backward: the model was not fitted with KSDF_FIT_ADJOINT");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  if (d_var_f && !m->adjoint_varf) {
    set_error("backward: a var_f cotangent needs a fit with KSDF_FIT_ADJOINT_VARF");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  const size_t fb = m->precision == KSDF_FP64 ? sizeof(double) : sizeof(float);
  const long nc = (long)m->n_cells + 1;
  char* w = static_cast<char*>(ws);
  double* part = reinterpret_cast<double*>(w);
  w += al256(2 * Q * sizeof(double));
  double* red = reinterpret_cast<double*>(w);
  w += al256(2 * RB * sizeof(double));
  int* key = reinterpret_cast<int*>(w);
  w += al256(Q * sizeof(int));
  int* perm = reinterpret_cast<int*>(w);
  w += al256(Q * sizeof(int));
  int* count = reinterpret_cast<int*>(w);
  w += al256(nc * sizeof(int));
  int* cursor = reinterpret_cast<int*>(w);
  w += al256(nc * sizeof(int));
  int* am = reinterpret_cast<int*>(w);
  w += al256(Q * sizeof(int));
  char* fwd = w;
  w += al256(Q * 5 * fb);
  void* fws = w;
  if (!argmin && Q > 0) {
    // recover each query's argmin cell with a forward pass into the workspace
    int r = launch_query(m, points, Q, sign, fwd, fwd + Q * fb, fwd + 4 * Q * fb, nullptr, nullptr,
                         am, nullptr, fws, query_workspace_bytes(m, Q), s);
    if (r != KSDF_OK) return r;
    argmin = am;
  }
  if (Q > 0 && m->precision != KSDF_FP64) {
    const unsigned gq = (unsigned)((Q + ST - 1) / ST);
    hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)((nc + ST - 1) / ST)), dim3(ST), 0, s, count,
                       nc, 0);
    hipLaunchKernelGGL(argmin_count_kernel, dim3(gq), dim3(ST), 0, s, argmin, Q, m->n_cells, key,
                       count);
    hipLaunchKernelGGL(scan_counts_kernel, dim3(1), dim3(1024), 0, s, count, (int)nc, cursor);
    hipLaunchKernelGGL(argmin_scatter_kernel, dim3(gq), dim3(ST), 0, s, Q, key, cursor, perm);
  }
  const unsigned grid = (unsigned)((Q + BT - 1) / BT);
  const bool varf = d_var_f != nullptr;
  const double two_l2 = 2.0 * m->ell * m->ell;
  if (m->precision == KSDF_FP64) {
    BwdArgs<double> A{};
    A.pts = static_cast<const double*>(points);
    A.Q = Q; A.sign = sign; A.argmin = argmin;
    A.d_mean = static_cast<const double*>(d_mean);
    A.d_grad = static_cast<const double*>(d_grad);
    A.d_var = static_cast<const double*>(d_var);
    A.d_var_f = static_cast<const double*>(d_var_f);
    A.d_points = static_cast<double*>(d_points);
    if (cost) {
      A.c_mean = static_cast<const double*>(cost->mean);
      A.c_var = static_cast<const double*>(cost->var);
      A.c_margin = cost->margin;
      A.c_kvar = cost->kvar;
      A.c_cost = static_cast<double*>(cost->cost);
    }
    A.part = part;
    A.n_cells = m->n_cells;
    A.offsets = m->offsets; A.loff = m->loff;
    A.ps = m->ps64; A.sv = m->sv64; A.L = m->L64; A.xi = m->xi64;
    A.D = m->adjoint_varf ? m->D64 : nullptr;
    A.centre64 = m->centre64; A.box = m->box32;
    A.ell = m->ell; A.two_l2 = two_l2; A.alpha = m->alpha;
    A.alpha_tied = m->alpha_tied; A.uniform_noise = !m->has_svar;
    timer_mark(m, KSDF_TIMER_BACKWARD, 0, s);
    if (Q > 0 && m->kernel == KSDF_KERNEL_MATERN32) {
      if (varf) hipLaunchKernelGGL((bwd_matern_kernel<double, true>), dim3(grid), dim3(BT), 0, s, A);
      else hipLaunchKernelGGL((bwd_matern_kernel<double, false>), dim3(grid), dim3(BT), 0, s, A);
    } else if (Q > 0) {
      if (varf) hipLaunchKernelGGL((bwd_plain_kernel<double, true>), dim3(grid), dim3(BT), 0, s, A);
      else hipLaunchKernelGGL((bwd_plain_kernel<double, false>), dim3(grid), dim3(BT), 0, s, A);
    }
    timer_mark(m, KSDF_TIMER_BACKWARD, 1, s);
  } else {
    BwdArgs<float> A{};
    A.pts = static_cast<const float*>(points);
    A.Q = Q; A.sign = sign; A.argmin = argmin;
    A.d_mean = static_cast<const float*>(d_mean);
    A.d_grad = static_cast<const float*>(d_grad);
    A.d_var = static_cast<const float*>(d_var);
    A.d_var_f = static_cast<const float*>(d_var_f);
    A.d_points = static_cast<float*>(d_points);
    if (cost) {
      A.c_mean = static_cast<const float*>(cost->mean);
      A.c_var = static_cast<const float*>(cost->var);
      A.c_margin = (float)cost->margin;
      A.c_kvar = (float)cost->kvar;
      A.c_cost = static_cast<float*>(cost->cost);
    }
    A.part = part;
    A.n_cells = m->n_cells;
    A.offsets = m->offsets; A.loff = m->loff;
    A.ps = m->ps32; A.sv = m->sv32; A.L = m->L32; A.xi = m->xi32;
    A.D = m->adjoint_varf ? m->D32 : nullptr;
    A.centre64 = m->centre64; A.box = m->box32;
    A.ell = (float)m->ell; A.two_l2 = (float)two_l2; A.alpha = (float)m->alpha;
    A.ell_d = m->ell; A.alpha_d = m->alpha; A.plo = m->plo32;
    {
      const double c2 = 1.4426950408889634 / two_l2;
      A.c2_ff[0] = (float)c2;
      A.c2_ff[1] = (float)(c2 - (double)A.c2_ff[0]);
      const double mc = std::sqrt(3.0) / m->ell, mcl = mc * 1.4426950408889634;
      A.mc_ff[0] = (float)mc;
      A.mc_ff[1] = (float)(mc - (double)A.mc_ff[0]);
      A.mcl_ff[0] = (float)mcl;
      A.mcl_ff[1] = (float)(mcl - (double)A.mcl_ff[0]);
    }
    A.alpha_tied = m->alpha_tied; A.uniform_noise = !m->has_svar;
    timer_mark(m, KSDF_TIMER_BACKWARD, 0, s);
    if (Q > 0 && m->kernel == KSDF_KERNEL_MATERN32) {
      if (varf) hipLaunchKernelGGL((bwd_matern_kernel<float, true>), dim3(grid), dim3(BT), 0, s, A);
      else hipLaunchKernelGGL((bwd_matern_kernel<float, false>), dim3(grid), dim3(BT), 0, s, A);
    } else if (Q > 0) {
      if (varf) hipLaunchKernelGGL((bwd_wave_kernel<true, false>), dim3(grid), dim3(BT), 0, s, A, perm);
      else if (m->tuning.backward_lanes)
        hipLaunchKernelGGL((bwd_wave_kernel<false, true>), dim3(grid), dim3(BT), 0, s, A, perm);
      else hipLaunchKernelGGL((bwd_wave_kernel<false, false>), dim3(grid), dim3(BT), 0, s, A, perm);
    }
    timer_mark(m, KSDF_TIMER_BACKWARD, 1, s);
  }
  if (m->precision == KSDF_FP64) {
    hipLaunchKernelGGL(theta_partial_kernel, dim3(RB), dim3(RT), 0, s, part, Q, red);
    hipLaunchKernelGGL(theta_final_kernel, dim3(1), dim3(RT), 0, s, red, d_hyper);
  } else {
    hipLaunchKernelGGL(theta_partial32_kernel, dim3(RB), dim3(RT), 0, s,
                       reinterpret_cast<const float2*>(part), Q, reinterpret_cast<float4*>(red));
    hipLaunchKernelGGL(theta_final32_kernel, dim3(1), dim3(RT), 0, s,
                       reinterpret_cast<const float4*>(red), d_hyper);
  }
  KSDF_HIP_TRY(hipGetLastError());
  return KSDF_OK;
}

}  // namespace ksdf
