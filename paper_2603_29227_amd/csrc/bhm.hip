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
// exponentials and n_h^3 multiply-adds instead of n_h^3 exponentials; the sum runs
// in FP64 (a sign is a decision: it is taken in double).
#include <cmath>

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
};

template <class T>
__device__ double bhm_logodds(const BhmArgs& A, const T* pts, long q, bool* have) {
  const double x[3] = {(double)pts[3 * q], (double)pts[3 * q + 1], (double)pts[3 * q + 2]};
  long key[3];
  for (int d = 0; d < 3; ++d) key[d] = (long)floor((x[d] - A.origin[d]) / A.box);
  *have = false;
  for (int d = 0; d < 3; ++d)
    if (key[d] < 0 || key[d] >= A.dims[d]) return 0.0;
  const long b = (key[0] * A.dims[1] + key[1]) * A.dims[2] + key[2];
  const int id = A.box_bhm[b];
  if (id < 0) return 0.0;
  *have = true;
  const int nh = A.nh;
  // per-axis factors exp(-gamma (x_d - h_d)^2), h_d = box corner + i * spacing
  double e[3][MAX_HINGES];
  for (int d = 0; d < 3; ++d) {
    const double lo = A.origin[d] + (double)key[d] * A.box;
    for (int i = 0; i < nh; ++i) {
      const double t = x[d] - (lo + (double)i * A.spacing);
      e[d][i] = exp(-A.gamma * t * t);
    }
  }
  const long m = (long)nh * nh * nh;
  const double* w = A.weights + (long)id * (m + 1);
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

template <class T>
__global__ void __launch_bounds__(BT) bhm_sign_kernel(BhmArgs A, const T* pts, long Q, double tau,
                                                      int8_t* sign, double* logodds) {
  const long q = (long)blockIdx.x * BT + threadIdx.x;
  if (q >= Q) return;
  bool have;
  const double l = bhm_logodds(A, pts, q, &have);
  // no local map: the box holds no occupied voxel, taken as free space
  sign[q] = (!have || l < tau) ? 1 : -1;
  if (logodds) logodds[q] = have ? l : -INFINITY;
}

// per-block sums of l at the hit points, in a fixed order (tree in LDS)
template <class T>
__global__ void __launch_bounds__(BT) bhm_tau_partial_kernel(BhmArgs A, const T* pts, long K,
                                                             double* part) {
  __shared__ double red[BT];
  const long q = (long)blockIdx.x * BT + threadIdx.x;
  double l = 0.0;
  if (q < K) {
    bool have;
    l = bhm_logodds(A, pts, q, &have);
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int o = BT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// tau <- (1 - alpha) tau + (alpha / K) sum_k l(x_k); the partial sums in block order
__global__ void __launch_bounds__(BT) bhm_tau_final_kernel(const double* part, long n_part, long K,
                                                           double alpha, double* tau) {
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
  const unsigned g = (unsigned)((Q + BT - 1) / BT);
  if (dtype == KSDF_DTYPE_F64)
    hipLaunchKernelGGL(bhm_sign_kernel<double>, dim3(g), dim3(BT), 0, s, A,
                       static_cast<const double*>(points), Q, tau, sign, logodds);
  else
    hipLaunchKernelGGL(bhm_sign_kernel<float>, dim3(g), dim3(BT), 0, s, A,
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
  hipLaunchKernelGGL(bhm_tau_final_kernel, dim3(1), dim3(BT), 0, s, part, g, K, alpha, tau);
  KSDF_HIP_TRY(hipGetLastError());
  return KSDF_OK;
}

}  // namespace ksdf
