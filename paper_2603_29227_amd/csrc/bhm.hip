// SDF sign from Bayesian-Hilbert-map weights (Sec. IV-A sign prediction, App. B).
//
// The occupancy log-odds of a local BHM is l(x) = mu^T phi(x) with features
// phi(x) = [k(x, h_1), ..., k(x, h_M), 1], k(x, h) = exp(-gamma |x - h|^2) over the
// hinge points h of the local map; the sign is +1 (free) where l(x) < tau and -1
// otherwise, and tau follows a moving average of the log-odds at hit points.
//
// Local maps sit on a lattice of boxes of edge B; each holds n_h^3 hinge points at
// the lattice points of its box (spacing B / (n_h - 1)) plus the bias feature.  A
// query uses the map of the box it lies in.  The RBF over a lattice separates by axis,
// k = exp(-gamma dx^2) exp(-gamma dy^2) exp(-gamma dz^2), so a query takes 3 n_h
// exponentials and n_h^3 multiply-adds instead of n_h^3 exponentials.  Double points
// are evaluated in FP64, float points in FP32 with a compensated outer sum (the
// decision l < tau is then the FP32 one).
#include <climits>
#include <cmath>

#include "ff.h"
#include "ksdf_internal.h"

namespace ksdf {
namespace {

constexpr int BT = 256;
constexpr int MAX_HINGES = 16;

struct BhmArgs {
  double origin[3];
  double box;
  double spacing;
  int dims[3];
  int nh;
  double gamma;
  const int* box_bhm;
  const double* weights;
  // float pairs of the layout for the FP32 evaluation
  float origin_ff[3][2];
  float box_ff[2];
  float spacing_ff[2];
};

// The map box of a point: its lattice key, the flat box index and the map id (-1: no
// map, or outside the lattice).
template <class T>
__device__ __forceinline__ int bhm_box(const BhmArgs& A, const T* pts, long q, long key[3]) {
  for (int d = 0; d < 3; ++d)
    key[d] = (long)floor(((double)pts[3 * q + d] - A.origin[d]) / A.box);
  for (int d = 0; d < 3; ++d)
    if (key[d] < 0 || key[d] >= A.dims[d]) return -1;
  return A.box_bhm[(key[0] * A.dims[1] + key[1]) * A.dims[2] + key[2]];
}

// Log-odds of a point in FP64 (double points): per-axis factors, then the separable sum.
__device__ double bhm_logodds64(const BhmArgs& A, const double* pts, long q, const long key[3],
                                const double* w) {
  const int nh = A.nh;
  double e[3][MAX_HINGES];
  for (int d = 0; d < 3; ++d) {
    const double lo = A.origin[d] + (double)key[d] * A.box;
    for (int i = 0; i < nh; ++i) {
      const double t = pts[3 * q + d] - (lo + (double)i * A.spacing);
      e[d][i] = exp(-A.gamma * t * t);
    }
  }
  const long m = (long)nh * nh * nh;
  double l = w[m];   // bias feature
  for (int i = 0; i < nh; ++i)
    for (int j = 0; j < nh; ++j) {
      const double eij = e[0][i] * e[1][j];
      const double* wr = w + ((long)i * nh + j) * nh;
      double acc = 0.0;
      for (int k = 0; k < nh; ++k) acc += wr[k] * e[2][k];
      l += eij * acc;
    }
  return l;
}

// The same for float points, in FP32: the offsets to the hinges from the exact
// difference of the point and the hinge coordinate (the hinge as a float pair), the
// factors from the FP32 exp, the inner sums over the last axis plain and the outer sum
// with TwoSum compensation.  The error is a few float roundings of sum |terms|; where
// |l - tau| is below that, the sign is the FP32 decision.
// The FP32 log-odds with the hinge count as a compile-time constant NH: every loop
// unrolls and the per-axis factors stay in registers.  The same operations in the same
// order as bhm_logodds32_any below.
template <int NH>
__device__ __forceinline__ float bhm_logodds32_t(const BhmArgs& A, const float* pts, long q,
                                                 const long key[3], const double* w) {
  float e[3][NH];
  const float g = (float)A.gamma;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    // x - (box corner) as a float pair, the corner origin + key B from the layout's pairs
    const ff lo = ff_add(ff{A.origin_ff[d][0], A.origin_ff[d][1]},
                         ff_mul_f(ff{A.box_ff[0], A.box_ff[1]}, (float)key[d]));
    const ff t0 = ff_add(ff{pts[3 * q + d], 0.f}, ff_neg(lo));
#pragma unroll
    for (int i = 0; i < NH; ++i) {
      const float fi = (float)i;
      const float tt = fmaf(-fi, A.spacing_ff[0], t0.hi) + fmaf(-fi, A.spacing_ff[1], t0.lo);
      e[d][i] = expf(-g * tt * tt);
    }
  }
  constexpr int m = NH * NH * NH;
  float s = (float)w[m], c = 0.f;   // bias feature; compensated outer sum
#pragma unroll
  for (int i = 0; i < NH; ++i)
#pragma unroll
    for (int j = 0; j < NH; ++j) {
      const float eij = e[0][i] * e[1][j];
      const double* wr = w + (i * NH + j) * NH;
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < NH; ++k) acc = fmaf((float)wr[k], e[2][k], acc);
      const ff p = ff_two_sum(s, eij * acc);
      s = p.hi;
      c += p.lo;
    }
  return s + c;
}

// Any hinge count (read from the layout; the factor arrays live in private memory).
__device__ float bhm_logodds32_any(const BhmArgs& A, const float* pts, long q, const long key[3],
                                   const double* w) {
  const int nh = A.nh;
  float e[3][MAX_HINGES];
  const float g = (float)A.gamma;
  for (int d = 0; d < 3; ++d) {
    const ff lo = ff_add(ff{A.origin_ff[d][0], A.origin_ff[d][1]},
                         ff_mul_f(ff{A.box_ff[0], A.box_ff[1]}, (float)key[d]));
    const ff t0 = ff_add(ff{pts[3 * q + d], 0.f}, ff_neg(lo));
    for (int i = 0; i < nh; ++i) {
      const float fi = (float)i;
      const float tt = fmaf(-fi, A.spacing_ff[0], t0.hi) + fmaf(-fi, A.spacing_ff[1], t0.lo);
      e[d][i] = expf(-g * tt * tt);
    }
  }
  const int m = nh * nh * nh;
  float s = (float)w[m], c = 0.f;
  for (int i = 0; i < nh; ++i)
    for (int j = 0; j < nh; ++j) {
      const float eij = e[0][i] * e[1][j];
      const double* wr = w + (i * nh + j) * nh;
      float acc = 0.f;
      for (int k = 0; k < nh; ++k) acc = fmaf((float)wr[k], e[2][k], acc);
      const ff p = ff_two_sum(s, eij * acc);
      s = p.hi;
      c += p.lo;
    }
  return s + c;
}

// 7 hinges per axis (the indoor setting) in registers; other counts the general form
__device__ __forceinline__ float bhm_logodds32(const BhmArgs& A, const float* pts, long q,
                                               const long key[3], const double* w) {
  if (A.nh == 7) return bhm_logodds32_t<7>(A, pts, q, key, w);
  return bhm_logodds32_any(A, pts, q, key, w);
}

// Points sorted by map box within each block (bitonic sort of (map id, slot) keys in
// LDS), so that a wave's points mostly share a map: a wave whose points all lie in one
// map reads its weights through wave-uniform (scalar) loads, and one that spans a few
// maps loads each weight from a few addresses.  A larger block lets a wave meet fewer
// maps but costs occupancy (on the 256^3 room grid, blocks of 128, 256, 512 and 1024
// points took 0.85, 0.58, 0.63 and 0.92 ms).  Each point's result goes back to its
// own index.
constexpr int BS = 256;
// Workgroups go to the 8 XCDs (each with its own L2) in turn; neighbouring blocks of
// points read the same maps, so each XCD takes one contiguous range of the blocks (a
// bijection of [0, n); the results do not depend on it).
__device__ __forceinline__ long bhm_block(long n) {
  constexpr long NX = 8;
  const long i = blockIdx.x, q = n / NX, r = n % NX;
  const long x = i % NX, k = i / NX;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}
template <class T>
__device__ __forceinline__ void bhm_sorted_slot(const BhmArgs& A, const T* pts, long Q, long* q_out,
                                                int* id_out) {
  __shared__ unsigned long long keys[BS];
  const long blk = bhm_block(gridDim.x);
  const long q = blk * BS + threadIdx.x;
  long key[3];
  const int id = q < Q ? bhm_box(A, pts, q, key) : INT_MAX - 1;
  keys[threadIdx.x] = ((unsigned long long)(unsigned)(id + 1) << 32) | threadIdx.x;
  for (int k = 2; k <= BS; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      __syncthreads();
      const int t = threadIdx.x, o = t ^ j;
      if (o > t) {
        const unsigned long long a = keys[t], b = keys[o];
        const bool up = (t & k) == 0;
        if ((a > b) == up) {
          keys[t] = b;
          keys[o] = a;
        }
      }
    }
  __syncthreads();
  const unsigned long long k = keys[threadIdx.x];
  *q_out = blk * BS + (long)(k & 0xffffffffu);
  *id_out = (int)(k >> 32) - 1;
}

template <class T>
__global__ void __launch_bounds__(BS) bhm_sign_kernel(BhmArgs A, const T* pts, long Q, double tau,
                                                      int8_t* sign, double* logodds) {
  long q;
  int id;
  bhm_sorted_slot(A, pts, Q, &q, &id);
  if (q >= Q) return;
  long key[3];
  bhm_box(A, pts, q, key);
  const long m = (long)A.nh * A.nh * A.nh;
  double l = 0.0;
  const bool have = id >= 0;
  if (have) {
    // one map for the whole wave: its weights through scalar loads
    const int w0 = __builtin_amdgcn_readfirstlane(id);
    const bool uni = __ballot(id != w0) == 0ull;
    const double* w = A.weights + (long)(uni ? w0 : id) * (m + 1);
    if constexpr (sizeof(T) == 8) l = bhm_logodds64(A, pts, q, key, w);
    else l = (double)bhm_logodds32(A, pts, q, key, w);
  }
  // no local map: the box holds no occupied voxel, taken as free space
  sign[q] = (!have || l < tau) ? 1 : -1;
  if (logodds) logodds[q] = have ? l : -INFINITY;
}

// per-block sums of l at the hit points, in a fixed order (tree in LDS): FP64 for
// double points; float-float for float points (the FP32 log-odds summed by TwoSum)
template <class T>
__global__ void __launch_bounds__(BT) bhm_tau_partial_kernel(BhmArgs A, const T* pts, long K,
                                                             double* part) {
  __shared__ double red[BT];
  __shared__ float rh[BT], rl[BT];
  const long q = (long)blockIdx.x * BT + threadIdx.x;
  double l = 0.0;
  float lf = 0.f;
  if (q < K) {
    long key[3];
    const int id = bhm_box(A, pts, q, key);
    if (id >= 0) {
      const double* w = A.weights + (long)id * ((long)A.nh * A.nh * A.nh + 1);
      if constexpr (sizeof(T) == 8) l = bhm_logodds64(A, pts, q, key, w);
      else lf = bhm_logodds32(A, pts, q, key, w);
    }
  }
  if constexpr (sizeof(T) == 8) {
    red[threadIdx.x] = l;
    __syncthreads();
    for (int o = BT / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
  } else {
    rh[threadIdx.x] = lf;
    rl[threadIdx.x] = 0.f;
    __syncthreads();
    for (int o = BT / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) {
        const ff a = ff_add(ff{rh[threadIdx.x], rl[threadIdx.x]},
                            ff{rh[threadIdx.x + o], rl[threadIdx.x + o]});
        rh[threadIdx.x] = a.hi;
        rl[threadIdx.x] = a.lo;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) reinterpret_cast<float2*>(part)[blockIdx.x] = make_float2(rh[0], rl[0]);
  }
}

// tau <- (1 - alpha) tau + (alpha / K) sum_k l(x_k), the partial sums in block order;
// FP64 for double points, float-float for float points (tau converted in and out)
template <bool F64>
__global__ void __launch_bounds__(BT) bhm_tau_final_kernel(const double* part, long n_part, long K,
                                                           double alpha, double* tau) {
  if constexpr (F64) {
    __shared__ double red[BT];
    double s = 0.0;
    for (long i = threadIdx.x; i < n_part; i += BT) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = BT / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) *tau = (1.0 - alpha) * *tau + alpha / (double)K * red[0];
  } else {
    __shared__ float rh[BT], rl[BT];
    const float2* pf = reinterpret_cast<const float2*>(part);
    ff s{0.f, 0.f};
    for (long i = threadIdx.x; i < n_part; i += BT) s = ff_add(s, ff{pf[i].x, pf[i].y});
    rh[threadIdx.x] = s.hi;
    rl[threadIdx.x] = s.lo;
    __syncthreads();
    for (int o = BT / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) {
        const ff a = ff_add(ff{rh[threadIdx.x], rl[threadIdx.x]},
                            ff{rh[threadIdx.x + o], rl[threadIdx.x + o]});
        rh[threadIdx.x] = a.hi;
        rl[threadIdx.x] = a.lo;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double t0 = *tau, wk = alpha / (double)K, keep = 1.0 - alpha;
      const float th = (float)t0, wh = (float)wk, kh = (float)keep;
      const ff t{th, (float)(t0 - (double)th)}, w{wh, (float)(wk - (double)wh)},
          kp{kh, (float)(keep - (double)kh)};
      const ff r = ff_add(ff_mul(kp, t), ff_mul(w, ff{rh[0], rl[0]}));
      *tau = (double)r.hi + (double)r.lo;
    }
  }
}
bool make_bhm_args(const ksdf_bhm_layout* L, const int* box_bhm, const double* weights, BhmArgs* A) {
  if (!L || !box_bhm || !weights || !(L->box > 0) || !std::isfinite(L->box) || !(L->gamma > 0) ||
      !std::isfinite(L->gamma) || L->hinges < 2 || L->hinges > MAX_HINGES || L->dims[0] < 1 ||
      L->dims[1] < 1 || L->dims[2] < 1)
    return false;
  for (int d = 0; d < 3; ++d) {
    if (!std::isfinite(L->origin[d])) return false;
    A->origin[d] = L->origin[d];
    A->dims[d] = L->dims[d];
  }
  A->box = L->box;
  A->spacing = L->box / (double)(L->hinges - 1);
  A->nh = L->hinges;
  A->gamma = L->gamma;
  A->box_bhm = box_bhm;
  A->weights = weights;
  auto split = [](double v, float out[2]) {
    out[0] = (float)v;
    out[1] = (float)(v - (double)out[0]);
  };
  for (int d = 0; d < 3; ++d) split(A->origin[d], A->origin_ff[d]);
  split(A->box, A->box_ff);
  split(A->spacing, A->spacing_ff);
  return true;
}

}  // namespace

size_t bhm_tau_workspace_bytes(long K) { return (size_t)((K + BT - 1) / BT + 1) * sizeof(double); }

int launch_bhm_sign(const ksdf_bhm_layout* L, const int* box_bhm, const double* weights,
                    const void* points, int dtype, long Q, double tau, int8_t* sign,
                    double* logodds, hipStream_t s) {
  BhmArgs A;
  if (!make_bhm_args(L, box_bhm, weights, &A) || Q < 0 || (Q > 0 && (!points || !sign)) ||
      !std::isfinite(tau) || (dtype != KSDF_DTYPE_F32 && dtype != KSDF_DTYPE_F64)) {
    set_error("ksdf_bhm_sign: invalid argument");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  if (Q == 0) return KSDF_OK;
  const unsigned g = (unsigned)((Q + BS - 1) / BS);
  if (dtype == KSDF_DTYPE_F64)
    hipLaunchKernelGGL(bhm_sign_kernel<double>, dim3(g), dim3(BS), 0, s, A,
                       static_cast<const double*>(points), Q, tau, sign, logodds);
  else
    hipLaunchKernelGGL(bhm_sign_kernel<float>, dim3(g), dim3(BS), 0, s, A,
                       static_cast<const float*>(points), Q, tau, sign, logodds);
  KSDF_HIP_TRY(hipGetLastError());
  return KSDF_OK;
}

int launch_bhm_update_tau(const ksdf_bhm_layout* L, const int* box_bhm, const double* weights,
                          const void* hits, int dtype, long K, double alpha, double* tau, void* ws,
                          size_t ws_bytes, hipStream_t s) {
  BhmArgs A;
  if (!make_bhm_args(L, box_bhm, weights, &A) || K < 1 || !hits || !tau || !(alpha > 0) ||
      alpha > 1 || (dtype != KSDF_DTYPE_F32 && dtype != KSDF_DTYPE_F64)) {
    set_error("ksdf_bhm_update_tau: invalid argument");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  if (!ws || ws_bytes < bhm_tau_workspace_bytes(K)) {
    set_error("ksdf_bhm_update_tau: workspace too small");
    return KSDF_ERR_WORKSPACE;
  }
  double* part = static_cast<double*>(ws);
  const long g = (K + BT - 1) / BT;
  if (dtype == KSDF_DTYPE_F64)
    hipLaunchKernelGGL(bhm_tau_partial_kernel<double>, dim3((unsigned)g), dim3(BT), 0, s, A,
                       static_cast<const double*>(hits), K, part);
  else
    hipLaunchKernelGGL(bhm_tau_partial_kernel<float>, dim3((unsigned)g), dim3(BT), 0, s, A,
                       static_cast<const float*>(hits), K, part);
  if (dtype == KSDF_DTYPE_F64)
    hipLaunchKernelGGL(bhm_tau_final_kernel<true>, dim3(1), dim3(BT), 0, s, part, g, K, alpha, tau);
  else
    hipLaunchKernelGGL(bhm_tau_final_kernel<false>, dim3(1), dim3(BT), 0, s, part, g, K, alpha, tau);
  KSDF_HIP_TRY(hipGetLastError());
  return KSDF_OK;
}

}  // namespace ksdf
