// Query forward, FP32 model: the per-point SDF prediction of Sec. IV-B laid out for
// 64-wide wavefronts.
//
// 1. Bucket.  Queries are counting-sorted by (Z-order rank of their candidate-index
//    box, Morton index of a sub-box of it) so the 64 queries of a wave sit in one
//    small region and mostly share their K nearest cells (Sec. IV-B.1, "K nearest
//    GPs"), also where queries are sparse.
// 2. Candidates.  Each lane keeps the K nearest occupied cell centres of its box's
//    list (fixed FP32 rounding sequence, ties by id).
// 3. Per-candidate UDF (eq. log_gp_posterior_mean with App. D scaling, Table I).
//    The wave walks the union of its lanes' candidates, nearest rank first; the cell
//    id is wave-uniform, so the cell's samples and weights come through scalar
//    loads and every lane that lists the cell evaluates it with full-rate FMAs and
//    one exp2 per sample.  Before a cell is walked each lane bounds its u from
//    below (sample bounding box and the sum of positive weights); if no lane can
//    improve on its current minimum, the cell is skipped, which does not change the
//    min-fusion result.
// 4. Near the surface the square root amplifies the FP32 error of u^2, and
//    ill-conditioned cells have strongly cancelling weights.  Each lane keeps an
//    error bound per cell from the cancellation ratio sum|a_i e_i| / |f'|; where
//    the bound could move the answer by more than a fraction of the tolerance, the
//    lane re-evaluates those cells in FP64.
// 5. Argmin cell.  The wave loops over the distinct argmin cells of its lanes (one
//    or two in practice): gradient w/|w|, GP variance 1 - |L^{-1} k*|^2 by forward
//    substitution with the factor rows in scalar registers, and the softmin
//    variance of Sec. IV-B.3 in one pass.
#include "query_dev.h"

namespace ksdf {
namespace {

template <int KM, int MB, int NT, bool MAT>
__global__ void __launch_bounds__(NT) query_fast_kernel(FastArgs A) {
  query_tile<KM, MB, MAT>(A, (long)blockIdx.x * NT + threadIdx.x);
}

template <int NT, bool MAT>
void launch_query_nt_k(const ksdf_model* m, const FastArgs& A, hipStream_t s) {
  const unsigned g = (unsigned)((A.Q + NT - 1) / NT);
  const bool k8 = m->k_fuse <= 8;
  const bool m64 = m->max_m <= 64;
  if (k8 && m64) hipLaunchKernelGGL((query_fast_kernel<8, 64, NT, MAT>), dim3(g), dim3(NT), 0, s, A);
  else if (k8) hipLaunchKernelGGL((query_fast_kernel<8, 128, NT, MAT>), dim3(g), dim3(NT), 0, s, A);
  else if (m64) hipLaunchKernelGGL((query_fast_kernel<16, 64, NT, MAT>), dim3(g), dim3(NT), 0, s, A);
  else hipLaunchKernelGGL((query_fast_kernel<16, 128, NT, MAT>), dim3(g), dim3(NT), 0, s, A);
}

template <int NT>
void launch_query_nt(const ksdf_model* m, const FastArgs& A, hipStream_t s) {
  if (A.matern) launch_query_nt_k<NT, true>(m, A, s);
  else launch_query_nt_k<NT, false>(m, A, s);
}

size_t bucketing_bytes(const ksdf_model* m, long Q) {
  const long nb = n_bins_of(m);
  const long tiles = (nb + SCAN_TILE - 1) / SCAN_TILE;
  return align256(Q * sizeof(int)) * 2 + align256(nb * sizeof(int)) * 2 +
         align256(tiles * sizeof(int));
}

}  // namespace

size_t query_fast_workspace_bytes(const ksdf_model* m, long Q) {
  const long nc = (long)m->n_cells + 1;
  const long tiles = (nc + SCAN_TILE - 1) / SCAN_TILE;
  const bool pairs = m->tuning.query_split && m->tuning.query_pairs && query_pairs_usable(m, Q);
  return bucketing_bytes(m, Q) + 2 * align256(Q * sizeof(P1Rec)) + 2 * align256(nc * sizeof(int)) +
         align256(tiles * sizeof(int)) + (pairs ? query_pairs_workspace_bytes(m, Q) : 0);
}

int launch_query_bucketing(const ksdf_model* m, const void* points, long Q, void* ws, hipStream_t s) {
  if (Q == 0) return KSDF_OK;
  FastArgs A = make_fast_args(m, points, Q, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                              nullptr, nullptr);
  return launch_bucketing(m, A, ws, s);
}

int launch_query_fast(const ksdf_model* m, const void* points, long Q, const int8_t* sign,
                      void* mean, void* grad, void* var, void* var_f, void* grad_var, int* argmin,
                      uint8_t* q_status, void* ws, size_t ws_bytes, hipStream_t s, bool prebucketed) {
  (void)ws_bytes;   // checked by the caller against query_workspace_bytes
  if (Q == 0) return KSDF_OK;
  FastArgs A = make_fast_args(m, points, Q, sign, mean, grad, var, var_f, grad_var, argmin, q_status);
  if (prebucketed) {
    A.perm = bucketed_perm(ws, Q);
  } else {
    int r = launch_bucketing(m, A, ws, s);
    if (r != KSDF_OK) return r;
  }
  timer_mark(m, KSDF_TIMER_QUERY, 0, s);
  if (m->tuning.query_split) {
    char* w = static_cast<char*>(ws) + bucketing_bytes(m, Q);
    const long nc = (long)m->n_cells + 1;
    P1Rec* rec = reinterpret_cast<P1Rec*>(w);
    w += align256(Q * sizeof(P1Rec));
    P1Rec* rec2 = reinterpret_cast<P1Rec*>(w);
    w += align256(Q * sizeof(P1Rec));
    int* count = reinterpret_cast<int*>(w);
    w += align256(nc * sizeof(int));
    int* cursor = reinterpret_cast<int*>(w);
    w += align256(nc * sizeof(int));
    int* tsum = reinterpret_cast<int*>(w);
    w += align256(((nc + SCAN_TILE - 1) / SCAN_TILE) * sizeof(int));
    void* pws = (m->tuning.query_pairs && query_pairs_usable(m, Q)) ? w : nullptr;
    if ((nc + SCAN_TILE - 1) / SCAN_TILE > (long)SCAN_TILE) {
      set_error("query: too many cells for the argmin regrouping");
      return KSDF_ERR_UNSUPPORTED;
    }
    const bool lane = m->tuning.query_lanes != 0;
    if (m->tuning.query_block == 64) {
      if (lane) launch_query_split_64_lane(m, A, rec, rec2, count, cursor, tsum, pws, s);
      else launch_query_split_64_wave(m, A, rec, rec2, count, cursor, tsum, pws, s);
    } else {
      if (lane) launch_query_split_256_lane(m, A, rec, rec2, count, cursor, tsum, pws, s);
      else launch_query_split_256_wave(m, A, rec, rec2, count, cursor, tsum, pws, s);
    }
  } else if (m->tuning.query_block == 64) {
    launch_query_nt<64>(m, A, s);
  } else {
    launch_query_nt<256>(m, A, s);
  }
  timer_mark(m, KSDF_TIMER_QUERY, 1, s);
  KSDF_HIP_TRY(hipGetLastError());
  return KSDF_OK;
}

}  // namespace ksdf
