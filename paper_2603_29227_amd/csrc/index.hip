// Candidate index for "the K nearest GPs" of Sec. IV-B.1.
//
// The fused cells of a query are the K occupied cells whose centres are nearest
// to it (ties by id).  The index partitions space into a lattice of cell-sized
// boxes.  For box B, D_K(B) is the K-th smallest, over occupied cells c, of the
// farthest distance from c's centre to B.  Every point of B then has K cells
// within D_K(B), so only cells whose nearest distance to B is <= D_K(B) can be
// among its K nearest; those cells (a superset, ascending ids) are B's list.  A
// query scans its box's list and keeps the K nearest exactly.
//
// One wave per box: lanes stride over the cells keeping a private sorted top-K of
// farthest distances, K rounds of a wave-wide min merge give D_K, and a ballot
// prefix writes the list in id order.  Built once per model (structure only), in
// two passes: the count pass fixes each box's list length (and so the list's size,
// which the caller then provides), the fill pass writes the lists.
#include <algorithm>
#include <cmath>
#include <utility>

#include "ksdf_internal.h"

namespace ksdf {
namespace {

constexpr int IDX_THREADS = 256;
constexpr int BOXES_PER_BLOCK = IDX_THREADS / 64;

struct IndexArgs {
  const double* centre;   // [n,3]
  int n_cells;
  int k;
  double origin[3];
  double h;
  int lo[3];
  int dims[3];
  long n_boxes;
  double* bound;          // [n_boxes] squared inclusion bound
  int* counts;            // [n_boxes]
  const int* off;         // [n_boxes+1] (fill pass)
  int* list;              // fill pass
};

__device__ __forceinline__ double wmin(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ void box_of(const IndexArgs& A, long b, double lo[3], double hi[3]) {
  const long i = b / ((long)A.dims[1] * A.dims[2]);
  const long j = (b / A.dims[2]) % A.dims[1];
  const long k = b % A.dims[2];
  const long key[3] = {A.lo[0] + i, A.lo[1] + j, A.lo[2] + k};
  for (int d = 0; d < 3; ++d) {
    lo[d] = A.origin[d] + (double)key[d] * A.h;
    hi[d] = A.origin[d] + (double)(key[d] + 1) * A.h;
  }
}

__global__ void __launch_bounds__(IDX_THREADS) index_count_kernel(IndexArgs A) {
  const long b = (long)blockIdx.x * BOXES_PER_BLOCK + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (b >= A.n_boxes) return;
  double lo[3], hi[3];
  box_of(A, b, lo, hi);
  double top[KSDF_MAX_K];
  for (int t = 0; t < KSDF_MAX_K; ++t) top[t] = INFINITY;
  for (int c = lane; c < A.n_cells; c += 64) {
    double far2 = 0;
    for (int d = 0; d < 3; ++d) {
      const double x = A.centre[3 * c + d];
      const double e = fmax(fabs(x - lo[d]), fabs(x - hi[d]));
      far2 += e * e;
    }
    // insert into the sorted private top-K
    if (far2 < top[A.k - 1]) {
      int t = A.k - 1;
      while (t > 0 && top[t - 1] > far2) { top[t] = top[t - 1]; --t; }
      top[t] = far2;
    }
  }
  // merge: K rounds of the wave-wide minimum of the private heads
  int head = 0;
  double dk = INFINITY;
  for (int r = 0; r < A.k; ++r) {
    const double mine = head < A.k ? top[head] : INFINITY;
    const double mn = wmin(mine);
    dk = mn;
    if (!(mn < INFINITY)) break;
    const unsigned long long who = __ballot(mine == mn);
    const int first = __ffsll((long long)who) - 1;
    if (lane == first) ++head;
  }
  // margins cover FP32 rounding of the query's box key and candidate distances
  const double bound = (dk < INFINITY) ? dk * (1.0 + 1e-5) + 1e-5 : INFINITY;
  int count = 0;
  for (int c0 = 0; c0 < A.n_cells; c0 += 64) {
    const int c = c0 + lane;
    bool in = false;
    if (c < A.n_cells) {
      double near2 = 0;
      for (int d = 0; d < 3; ++d) {
        const double x = A.centre[3 * c + d];
        const double e = fmax(fmax(lo[d] - x, 0.0), x - hi[d]);
        near2 += e * e;
      }
      in = near2 <= bound;
    }
    count += __popcll(__ballot(in));
  }
  if (lane == 0) {
    A.bound[b] = bound;
    A.counts[b] = count;
  }
}

__global__ void __launch_bounds__(IDX_THREADS) index_fill_kernel(IndexArgs A) {
  const long b = (long)blockIdx.x * BOXES_PER_BLOCK + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (b >= A.n_boxes) return;
  double lo[3], hi[3];
  box_of(A, b, lo, hi);
  const double bound = A.bound[b];
  int pos = A.off[b];
  for (int c0 = 0; c0 < A.n_cells; c0 += 64) {
    const int c = c0 + lane;
    bool in = false;
    if (c < A.n_cells) {
      double near2 = 0;
      for (int d = 0; d < 3; ++d) {
        const double x = A.centre[3 * c + d];
        const double e = fmax(fmax(lo[d] - x, 0.0), x - hi[d]);
        near2 += e * e;
      }
      in = near2 <= bound;
    }
    const unsigned long long bal = __ballot(in);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (in) A.list[pos + before] = c;
    pos += __popcll(bal);
  }
}

}  // namespace

int index_lattice(ksdf_model* m, const double* qlo, const double* qhi) {
  CandidateIndex& X = m->index;
  // lattice: occupied keys padded by two boxes, grown to cover the query box
  long klo[3] = {0, 0, 0}, khi[3] = {0, 0, 0};
  for (int d = 0; d < 3; ++d) {
    klo[d] = LONG_MAX;
    khi[d] = LONG_MIN;
  }
  for (int c = 0; c < m->n_cells; ++c)
    for (int d = 0; d < 3; ++d) {
      const long k = (long)std::floor((m->h_centre[3 * c + d] - m->origin[d]) / m->h);
      klo[d] = std::min(klo[d], k - 2);
      khi[d] = std::max(khi[d], k + 2);
    }
  if (qlo && qhi)
    for (int d = 0; d < 3; ++d) {
      klo[d] = std::min(klo[d], (long)std::floor((qlo[d] - m->origin[d]) / m->h));
      khi[d] = std::max(khi[d], (long)std::floor((qhi[d] - m->origin[d]) / m->h));
    }
  long n_boxes = 1;
  for (int d = 0; d < 3; ++d) {
    X.lo[d] = m->n_cells ? (int)klo[d] : 0;
    X.dims[d] = m->n_cells ? (int)(khi[d] - klo[d] + 1) : 0;
    n_boxes *= X.dims[d];
  }
  if (m->n_cells == 0 || n_boxes > (64L << 20)) {
    if (m->n_cells != 0) {
      set_error("candidate index lattice too large; narrow the query box");
      return KSDF_ERR_UNSUPPORTED;
    }
    n_boxes = 0;
  }
  X.n_boxes = n_boxes;
  return KSDF_OK;
}

namespace {
IndexArgs index_args(const ksdf_model* m) {
  const CandidateIndex& X = m->index;
  IndexArgs A{};
  A.centre = m->centre64;
  A.n_cells = m->n_cells;
  A.k = std::min(m->k_fuse, m->n_cells);
  for (int d = 0; d < 3; ++d) {
    A.origin[d] = m->origin[d];
    A.lo[d] = X.lo[d];
    A.dims[d] = X.dims[d];
  }
  A.h = m->h;
  A.n_boxes = X.n_boxes;
  A.bound = X.bound;
  A.counts = X.counts;
  A.off = X.box_off;
  A.list = X.box_list;
  return A;
}
}  // namespace

int index_count(ksdf_model* m, hipStream_t s) {
  CandidateIndex& X = m->index;
  const long n_boxes = X.n_boxes;
  X.entries = 0;
  X.max_list = 0;
  if (n_boxes == 0) return KSDF_OK;
  IndexArgs A = index_args(m);
  const unsigned grid = (unsigned)((n_boxes + BOXES_PER_BLOCK - 1) / BOXES_PER_BLOCK);
  hipLaunchKernelGGL(index_count_kernel, dim3(grid), dim3(IDX_THREADS), 0, s, A);
  KSDF_HIP_TRY(hipGetLastError());
  std::vector<int> cnt(n_boxes);
  KSDF_HIP_TRY(hipMemcpyAsync(cnt.data(), X.counts, n_boxes * sizeof(int), hipMemcpyDeviceToHost, s));
  KSDF_HIP_TRY(hipStreamSynchronize(s));
  std::vector<int> off(n_boxes + 1, 0);
  long total = 0;
  int mx = 0;
  for (long b = 0; b < n_boxes; ++b) {
    off[b] = (int)total;
    total += cnt[b];
    mx = std::max(mx, cnt[b]);
  }
  if (total > INT32_MAX) {
    set_error("candidate index too large");
    return KSDF_ERR_UNSUPPORTED;
  }
  off[n_boxes] = (int)total;
  X.entries = total;
  X.max_list = mx;
  // Z-order rank of every box: query bucketing orders its bins by it, so that the
  // queries of one wave stay spatially compact also where they are sparse
  std::vector<std::pair<uint64_t, int>> z(n_boxes);
  for (long b = 0; b < n_boxes; ++b) {
    const long bx = b % X.dims[0], by = (b / X.dims[0]) % X.dims[1], bz = b / ((long)X.dims[0] * X.dims[1]);
    uint64_t code = 0;
    for (int bit = 0; bit < 21; ++bit)
      code |= (((uint64_t)(bx >> bit) & 1) << (3 * bit)) | (((uint64_t)(by >> bit) & 1) << (3 * bit + 1)) |
              (((uint64_t)(bz >> bit) & 1) << (3 * bit + 2));
    z[b] = {code, (int)b};
  }
  std::sort(z.begin(), z.end());
  std::vector<int> rank(n_boxes);
  for (long r = 0; r < n_boxes; ++r) rank[z[r].second] = (int)r;
  KSDF_HIP_TRY(hipMemcpyAsync(X.box_off, off.data(), (n_boxes + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  KSDF_HIP_TRY(hipMemcpyAsync(X.box_rank, rank.data(), n_boxes * sizeof(int), hipMemcpyHostToDevice, s));
  // the host vectors go out of scope on return
  KSDF_HIP_TRY(hipStreamSynchronize(s));
  return KSDF_OK;
}

int index_fill(ksdf_model* m, hipStream_t s) {
  if (m->index.n_boxes == 0) return KSDF_OK;
  IndexArgs A = index_args(m);
  const unsigned grid = (unsigned)((m->index.n_boxes + BOXES_PER_BLOCK - 1) / BOXES_PER_BLOCK);
  hipLaunchKernelGGL(index_fill_kernel, dim3(grid), dim3(IDX_THREADS), 0, s, A);
  KSDF_HIP_TRY(hipGetLastError());
  return KSDF_OK;
}

}  // namespace ksdf
