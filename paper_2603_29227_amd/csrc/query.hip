// Query forward: the per-point SDF prediction of Sec. IV-B.
//
// For each query x*: the K nearest occupied cell centres (ties by id); for each of
// them the log-GP mean with App. D scaling, f' = sum_i a_i exp(-(z_i^2 - d^2)/2l^2)
// and u_c = sqrt(d^2 - 2 l^2 ln f') (Table I; f' <= 0 excludes the cell, u^2 < 0
// clamps to 0); min-fusion u = min_c u_c (ties to the lowest id); then, on the
// argmin cell, the UDF gradient w/|w| with w = sum_i a_i e_i (x* - x_i), the GP
// variance 1 - |L^{-1} k*|^2 by forward substitution, and the softmin variance
// sum_i c_i^2 sigma_i^2, c_i = s_i (alpha h - alpha z_i + 1).  d = s u (sign input).
//
// The Matern 3/2 kernel of Table I replaces k by (1 + c r) exp(-c r), c = sqrt(3)/l,
// the transform by u = d - ln(f')/c (App. D scaling gamma = exp(c d)) and e_i in w
// by exp(-c (z_i - d)), since dk/dr = -c^2 r exp(-c r); u < 0 clamps to 0.
//
// This file holds the plain path: one thread per query, every read straight from
// the per-cell store (no staging, no bucketing), in the model's precision.  It serves
// FP64 models and FP32 Matern models; FP32 RBF models use the wave-cooperative
// kernels of query_fast.hip.
#include <cmath>

#include "ksdf_internal.h"

namespace ksdf {

template <class T>
struct QueryArgs {
  const T* pts;
  long Q;
  const int8_t* sign;
  T* mean;
  T* grad;
  T* var;
  T* var_f;
  T* grad_var;
  int* argmin;
  uint8_t* qst;
  int n_cells;
  int k;
  const int* offsets;
  const long* loff;
  const T* ps;        // [nnz,4] (px,py,pz,a) cell-local
  const T* sv;        // [nnz]
  const T* L;         // packed rows, reciprocal diagonal
  const float* centre32;
  const double* centre64;
  double origin[3];
  double h;
  int lo[3];
  int dims[3];
  long n_boxes;
  const int* box_off;
  const int* box_list;
  T inv2l2;           // 1/(2 l^2)
  T two_l2;           // 2 l^2
  T alpha;            // softmin temperature
  int kernel;         // KSDF_KERNEL_*
  T mc;               // Matern 3/2 rate sqrt(3) / l
};

namespace {

constexpr int QT = 256;

// Candidate distances: an integer decision, so both precisions use a fixed
// rounding sequence (float: sub, mul, two fma; double: sub, mul, add in order).
__device__ __forceinline__ float cand_d2(float qx, float qy, float qz, const float* c) {
  const float dx = __fsub_rn(qx, c[0]), dy = __fsub_rn(qy, c[1]), dz = __fsub_rn(qz, c[2]);
  float t = __fmul_rn(dx, dx);
  t = __fmaf_rn(dy, dy, t);
  return __fmaf_rn(dz, dz, t);
}
__device__ __forceinline__ double cand_d2(double qx, double qy, double qz, const double* c) {
  const double dx = __dsub_rn(qx, c[0]), dy = __dsub_rn(qy, c[1]), dz = __dsub_rn(qz, c[2]);
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}
template <class T> __device__ __forceinline__ const T* centre_of(const QueryArgs<T>& A, int c);
template <> __device__ __forceinline__ const float* centre_of(const QueryArgs<float>& A, int c) {
  return A.centre32 + 4L * c;
}
template <> __device__ __forceinline__ const double* centre_of(const QueryArgs<double>& A, int c) {
  return A.centre64 + 3L * c;
}

template <class T>
__device__ int select_candidates(const QueryArgs<T>& A, T qx, T qy, T qz, int* cid, bool* outside) {
  T cd[KSDF_MAX_K];
  int n = 0;
  const long key[3] = {(long)floor(((double)qx - A.origin[0]) / A.h) - A.lo[0],
                       (long)floor(((double)qy - A.origin[1]) / A.h) - A.lo[1],
                       (long)floor(((double)qz - A.origin[2]) / A.h) - A.lo[2]};
  const bool inside = A.n_boxes > 0 && key[0] >= 0 && key[0] < A.dims[0] && key[1] >= 0 &&
                      key[1] < A.dims[1] && key[2] >= 0 && key[2] < A.dims[2];
  *outside = !inside;
  int beg = 0, end = A.n_cells;
  const int* list = nullptr;
  if (inside) {
    const long b = (key[0] * A.dims[1] + key[1]) * A.dims[2] + key[2];
    beg = A.box_off[b];
    end = A.box_off[b + 1];
    list = A.box_list;
  }
  for (int t = beg; t < end; ++t) {
    const int c = list ? list[t] : t;
    const T d2 = cand_d2(qx, qy, qz, centre_of(A, c));
    if (n < A.k || d2 < cd[n - 1]) {   // ids ascend, so an equal distance never displaces
      int j = n < A.k ? n++ : n - 1;
      while (j > 0 && cd[j - 1] > d2) {
        cd[j] = cd[j - 1];
        cid[j] = cid[j - 1];
        --j;
      }
      cd[j] = d2;
      cid[j] = c;
    }
  }
  return n;
}

template <class T>
__device__ T cell_udf(const QueryArgs<T>& A, int c, T qx, T qy, T qz, bool* clamped) {
  const int b = A.offsets[c], m = A.offsets[c + 1] - b;
  const double* cc = A.centre64 + 3L * c;
  const T lx = qx - (T)cc[0], ly = qy - (T)cc[1], lz = qz - (T)cc[2];
  const T* p = A.ps + 4L * b;
  T d2 = (T)INFINITY;
  for (int i = 0; i < m; ++i) {
    const T dx = lx - p[4 * i], dy = ly - p[4 * i + 1], dz = lz - p[4 * i + 2];
    d2 = min(d2, dx * dx + dy * dy + dz * dz);
  }
  T f = T(0);
  *clamped = false;
  if (A.kernel == KSDF_KERNEL_MATERN32) {
    const T d = sqrt(d2);
    for (int i = 0; i < m; ++i) {
      const T dx = lx - p[4 * i], dy = ly - p[4 * i + 1], dz = lz - p[4 * i + 2];
      const T z = sqrt(dx * dx + dy * dy + dz * dz);
      f += p[4 * i + 3] * (T(1) + A.mc * z) * exp(-A.mc * (z - d));
    }
    if (!(f > T(0))) return (T)INFINITY;
    const T u = d - log(f) / A.mc;
    if (u < T(0)) {
      *clamped = true;
      return T(0);
    }
    return u;
  }
  for (int i = 0; i < m; ++i) {
    const T dx = lx - p[4 * i], dy = ly - p[4 * i + 1], dz = lz - p[4 * i + 2];
    const T z2 = dx * dx + dy * dy + dz * dz;
    f += p[4 * i + 3] * exp(-(z2 - d2) * A.inv2l2);
  }
  if (!(f > T(0))) return (T)INFINITY;
  const T u2 = d2 - A.two_l2 * log(f);
  if (u2 < T(0)) {
    *clamped = true;
    return T(0);
  }
  return sqrt(u2);
}

template <class T>
__global__ void __launch_bounds__(QT) query_plain_kernel(QueryArgs<T> A) {
  const long q = (long)blockIdx.x * QT + threadIdx.x;
  if (q >= A.Q) return;
  const T qx = A.pts[3 * q], qy = A.pts[3 * q + 1], qz = A.pts[3 * q + 2];
  const T sgn = A.sign ? (T)A.sign[q] : T(1);
  int cid[KSDF_MAX_K];
  bool outside = false;
  const int n = select_candidates(A, qx, qy, qz, cid, &outside);
  T best = (T)INFINITY;
  int bc = -1;
  bool bclamp = false;
  for (int t = 0; t < n; ++t) {
    bool cl;
    const T u = cell_udf(A, cid[t], qx, qy, qz, &cl);
    if (u < best || (u == best && u < (T)INFINITY && cid[t] < bc)) {
      best = u;
      bc = cid[t];
      bclamp = cl;
    }
  }
  uint8_t st = outside ? KSDF_Q_OUTSIDE_INDEX : 0;
  if (bc < 0) {
    A.mean[q] = (T)INFINITY;
    for (int d = 0; d < 3; ++d) A.grad[3 * q + d] = T(0);
    A.var[q] = (T)INFINITY;
    if (A.var_f) A.var_f[q] = T(1);
    if (A.grad_var)
      for (int d = 0; d < 3; ++d) A.grad_var[3 * q + d] = (T)INFINITY;
    if (A.argmin) A.argmin[q] = -1;
    if (A.qst) A.qst[q] = st | KSDF_Q_NO_VALID_CELL;
    return;
  }
  if (bclamp) st |= KSDF_Q_CLAMPED;
  // argmin cell: gradient, GP variance, softmin variance
  const int b = A.offsets[bc], m = A.offsets[bc + 1] - b;
  const double* cc = A.centre64 + 3L * bc;
  const T lx = qx - (T)cc[0], ly = qy - (T)cc[1], lz = qz - (T)cc[2];
  const T* p = A.ps + 4L * b;
  const T* sv = A.sv + b;
  const T* L = A.L + A.loff[bc];
  T d2 = (T)INFINITY;
  for (int i = 0; i < m; ++i) {
    const T dx = lx - p[4 * i], dy = ly - p[4 * i + 1], dz = lz - p[4 * i + 2];
    d2 = min(d2, dx * dx + dy * dy + dz * dz);
  }
  T w0 = 0, w1 = 0, w2 = 0;
  T v[KSDF_MAX_M];
  T vv = T(0);
  const T g = exp(-d2 * A.inv2l2);   // 1/gamma: k_i = e_i / gamma
  const T zmin = sqrt(d2);
  T S = 0, H = 0;
  const bool matern = A.kernel == KSDF_KERNEL_MATERN32;
  for (int i = 0; i < m; ++i) {
    const T dx = lx - p[4 * i], dy = ly - p[4 * i + 1], dz = lz - p[4 * i + 2];
    const T z2 = dx * dx + dy * dy + dz * dz;
    const T z = sqrt(z2);
    // e_i of the gradient (scaled) and the unscaled kernel value k_i
    T e, t;
    if (matern) {
      e = exp(-A.mc * (z - zmin));
      t = (T(1) + A.mc * z) * exp(-A.mc * z);
    } else {
      e = exp(-(z2 - d2) * A.inv2l2);
      t = e * g;
    }
    const T ae = p[4 * i + 3] * e;
    w0 += ae * dx;
    w1 += ae * dy;
    w2 += ae * dz;
    // forward substitution L v = k
    const T* row = L + (long)i * (i + 1) / 2;
    for (int j = 0; j < i; ++j) t -= row[j] * v[j];
    v[i] = t * row[i];
    vv += v[i] * v[i];
    const T s = exp(-A.alpha * (z - zmin));
    S += s;
    H += s * z;
  }
  const T h = H / S;
  T var = 0;
  // sums for the gradient variance: Vs = sum s_i v_i, g = sum l_i v_i (l_i = c_i)
  T Vs[3] = {0, 0, 0}, gs[3] = {0, 0, 0};
  for (int i = 0; i < m; ++i) {
    const T dx = lx - p[4 * i], dy = ly - p[4 * i + 1], dz = lz - p[4 * i + 2];
    const T z = sqrt(dx * dx + dy * dy + dz * dz);
    const T s = exp(-A.alpha * (z - zmin)) / S;
    const T ci = s * (A.alpha * h - A.alpha * z + T(1));
    var += ci * ci * sv[i];
    if (z > T(0)) {
      const T vd[3] = {dx / z, dy / z, dz / z};
      for (int d = 0; d < 3; ++d) {
        Vs[d] += s * vd[d];
        gs[d] += ci * vd[d];
      }
    }
  }
  if (A.grad_var) {
    // V[grad_k u] = sum_i sigma_i^2 |row k of J_i|^2 with J_i the derivative of the
    // softmin gradient g with respect to sample i (App. C):
    //   J_i = alpha w_i v_i^T + (l_i / z_i)(v_i v_i^T - I),
    //   w_i = l_i (v_i - Vs) + s_i (v_i - g).
    // As |v_i| = 1 the cross term of row k vanishes and
    //   |row k|^2 = alpha^2 w_ik^2 + (l_i / z_i)^2 (1 - v_ik^2).
    T gv[3] = {0, 0, 0};
    for (int i = 0; i < m; ++i) {
      const T dx = lx - p[4 * i], dy = ly - p[4 * i + 1], dz = lz - p[4 * i + 2];
      const T z = sqrt(dx * dx + dy * dy + dz * dz);
      if (!(z > T(0))) continue;   // a sample at the query has no direction
      const T s = exp(-A.alpha * (z - zmin)) / S;
      const T li = s * (A.alpha * h - A.alpha * z + T(1));
      const T vd[3] = {dx / z, dy / z, dz / z};
      const T lz2 = (li / z) * (li / z);
      for (int d = 0; d < 3; ++d) {
        const T w = li * (vd[d] - Vs[d]) + s * (vd[d] - gs[d]);
        gv[d] += sv[i] * (A.alpha * A.alpha * w * w + lz2 * (T(1) - vd[d] * vd[d]));
      }
    }
    for (int d = 0; d < 3; ++d) A.grad_var[3 * q + d] = gv[d];
  }
  const T wn = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
  T gx = 0, gy = 0, gz = 0;
  if (wn > T(0)) {
    gx = w0 / wn;
    gy = w1 / wn;
    gz = w2 / wn;
  } else {
    st |= KSDF_Q_GRAD_ZERO;
  }
  A.mean[q] = sgn * best;
  A.grad[3 * q] = sgn * gx;
  A.grad[3 * q + 1] = sgn * gy;
  A.grad[3 * q + 2] = sgn * gz;
  A.var[q] = var;
  if (A.var_f) A.var_f[q] = max(T(1) - vv, T(0));
  if (A.argmin) A.argmin[q] = bc;
  if (A.qst) A.qst[q] = st;
}

template <class T>
QueryArgs<T> make_args(const ksdf_model* m, const void* points, long Q, const int8_t* sign,
                       void* mean, void* grad, void* var, void* var_f, void* grad_var, int* argmin,
                       uint8_t* q_status) {
  QueryArgs<T> A{};
  A.pts = static_cast<const T*>(points);
  A.Q = Q;
  A.sign = sign;
  A.mean = static_cast<T*>(mean);
  A.grad = static_cast<T*>(grad);
  A.var = static_cast<T*>(var);
  A.var_f = static_cast<T*>(var_f);
  A.grad_var = static_cast<T*>(grad_var);
  A.argmin = argmin;
  A.qst = q_status;
  A.n_cells = m->n_cells;
  A.k = std::min(m->k_fuse, m->n_cells);
  A.offsets = m->offsets;
  A.loff = m->loff;
  A.centre32 = m->centre32;
  A.centre64 = m->centre64;
  for (int d = 0; d < 3; ++d) {
    A.origin[d] = m->origin[d];
    A.lo[d] = m->index.lo[d];
    A.dims[d] = m->index.dims[d];
  }
  A.h = m->h;
  A.n_boxes = m->index.n_boxes;
  A.box_off = m->index.box_off;
  A.box_list = m->index.box_list;
  A.inv2l2 = (T)(1.0 / (2.0 * m->ell * m->ell));
  A.two_l2 = (T)(2.0 * m->ell * m->ell);
  A.alpha = (T)m->alpha;
  A.kernel = m->kernel;
  A.mc = (T)(std::sqrt(3.0) / m->ell);
  return A;
}

}  // namespace

size_t query_workspace_bytes(const ksdf_model* m, long Q) {
  return m->precision == KSDF_FP32 ? query_fast_workspace_bytes(m, Q) : 0;
}

int launch_query(const ksdf_model* m, const void* points, long Q, const int8_t* sign, void* mean,
                 void* grad, void* var, void* var_f, void* grad_var, int* argmin, uint8_t* q_status, void* ws,
                 size_t ws_bytes, hipStream_t s, bool prebucketed) {
  if (Q == 0) return KSDF_OK;
  const unsigned grid = (unsigned)((Q + QT - 1) / QT);
  if (m->precision == KSDF_FP64) {
    QueryArgs<double> A = make_args<double>(m, points, Q, sign, mean, grad, var, var_f, grad_var, argmin, q_status);
    A.ps = m->ps64;
    A.sv = m->sv64;
    A.L = m->L64;
    timer_mark(m, KSDF_TIMER_QUERY, 0, s);
    hipLaunchKernelGGL(query_plain_kernel<double>, dim3(grid), dim3(QT), 0, s, A);
    timer_mark(m, KSDF_TIMER_QUERY, 1, s);
  } else {
    return launch_query_fast(m, points, Q, sign, mean, grad, var, var_f, grad_var, argmin, q_status, ws,
                             ws_bytes, s, prebucketed);
  }
  KSDF_HIP_TRY(hipGetLastError());
  return KSDF_OK;
}

}  // namespace ksdf
