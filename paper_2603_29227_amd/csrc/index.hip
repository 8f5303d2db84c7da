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
// Cell centres sit at the middle of lattice boxes, so both distances depend only on
// the integer key offset t between cell and box: per axis the centre lies t + 1/2
// edges from the box's low face, the far face is |t| + 1/2 edges away and the near
// one max(|t| - 1/2, 0).  In units of (h/2)^2 the squared distances are sums of odd
// squares, computed exactly in integers.  A cell outside a list is then at least
// one unit, (h/2)^2, farther from every point of the box than D_K(B); the bound
// keeps a margin for the FP32 rounding of the query's own distances.
//
// One wave per box, reading a dense map from lattice key to cell id.  D_K comes from
// shells of growing Chebyshev radius r around the box (24 r^2 + 2 keys each): lanes
// keep private sorted top-K lists of far distances, and after each shell K rounds of
// a wave-wide min merge give the K-th smallest so far; a cell in a later shell is at
// least (2r + 3)^2 + 2 units away, so once the K-th smallest is within that, it is
// final.  The list is then the cube of keys that can lie within the bound, scanned in
// key order (which is id order) with a ballot prefix for the writes.  Built once per
// model (structure only), in two passes: the count pass fixes each box's list length
// (and so the list's size, which the caller then provides), the fill pass writes the
// lists.
#include <algorithm>
#include <climits>
#include <cmath>
#include <utility>

#include "ksdf_internal.h"

namespace ksdf {
namespace {

constexpr int IDX_THREADS = 256;
constexpr int BOXES_PER_BLOCK = IDX_THREADS / 64;

struct IndexArgs {
  const int* kmap;        // [n_boxes] cell id at each lattice key, -1 where none
  int k;
  int dims[3];
  long n_boxes;
  float margin_abs;       // absolute rounding margin per sqrt(unit) of the bound
  long* bound;            // [n_boxes] inclusion bound on the near distance, (h/2)^2 units
  int* counts;            // [n_boxes]
  const int* off;         // [n_boxes+1] (fill pass)
  int* list;              // fill pass
};

// squared far / near distance along one axis, in (h/2)^2 units, for key offset |t| = a
__device__ __forceinline__ long far_units(int a) {
  const long v = 2L * a + 1;
  return v * v;
}
__device__ __forceinline__ long near_units(int a) {
  const long v = a > 0 ? 2L * a - 1 : 0;
  return v * v;
}

__device__ __forceinline__ long wmin_long(long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const long w = __shfl_xor(v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}

// The key offset of entry idx of shell r (keys at Chebyshev distance r from the box):
// the faces z = -r, +r (x, y in [-r, r]), y = -r, +r (|z| < r), x = -r, +r (|y|, |z| < r).
__device__ __forceinline__ void shell_key(int r, int idx, int& dx, int& dy, int& dz) {
  if (r == 0) {
    dx = dy = dz = 0;
    return;
  }
  const int n = 2 * r + 1, m = 2 * r - 1;
  if (idx < 2 * n * n) {
    const int e = idx % (n * n);
    dz = idx < n * n ? -r : r;
    dx = e / n - r;
    dy = e % n - r;
    return;
  }
  idx -= 2 * n * n;
  if (idx < 2 * n * m) {
    const int e = idx % (n * m);
    dy = idx < n * m ? -r : r;
    dx = e / m - r;
    dz = e % m - (r - 1);
    return;
  }
  idx -= 2 * n * m;
  const int e = idx % (m * m);
  dx = idx < m * m ? -r : r;
  dy = e / m - (r - 1);
  dz = e % m - (r - 1);
}

__device__ __forceinline__ void box_coords(const IndexArgs& A, long b, int& i, int& j, int& k) {
  i = (int)(b / ((long)A.dims[1] * A.dims[2]));
  j = (int)((b / A.dims[2]) % A.dims[1]);
  k = (int)(b % A.dims[2]);
}

// The cube of lattice keys around box (i, j, k) that can hold cells within `bound`
// (a key at Chebyshev distance r is at least (2r - 1)^2 units away), clipped to the
// lattice: low corner and extents.
__device__ __forceinline__ void bound_cube(const IndexArgs& A, int i, int j, int k, long bound,
                                           int lo[3], int n[3]) {
  const int reach = max(max(A.dims[0], A.dims[1]), A.dims[2]);
  int R = min((int)((sqrtf((float)bound) + 1.f) * 0.5f), reach);
  while (R < reach && near_units(R + 1) <= bound) ++R;
  while (R > 0 && near_units(R) > bound) --R;
  const int c[3] = {i, j, k};
  for (int d = 0; d < 3; ++d) {
    lo[d] = max(c[d] - R, 0);
    n[d] = min(c[d] + R, A.dims[d] - 1) - lo[d] + 1;
  }
}

// Visits the cube's keys in key order, lanes striding; f(id, in) for each batch of 64
// entries, `in` true where the key holds a cell whose near distance is within bound.
template <class F>
__device__ __forceinline__ void scan_cube(const IndexArgs& A, int i, int j, int k, long bound,
                                          F&& f) {
  int lo[3], n[3];
  bound_cube(A, i, j, k, bound, lo, n);
  const long vol = (long)n[0] * n[1] * n[2];
  const int lane = threadIdx.x & 63;
  for (long e0 = 0; e0 < vol; e0 += 64) {
    const long e = e0 + lane;
    int c = -1;
    if (e < vol) {
      const int x = lo[0] + (int)(e / ((long)n[1] * n[2]));
      const int y = lo[1] + (int)((e / n[2]) % n[1]);
      const int z = lo[2] + (int)(e % n[2]);
      const long near2 = near_units(abs(x - i)) + near_units(abs(y - j)) + near_units(abs(z - k));
      if (near2 <= bound) c = A.kmap[((long)x * A.dims[1] + y) * A.dims[2] + z];
    }
    f(c, c >= 0);
  }
}

__global__ void __launch_bounds__(IDX_THREADS) index_count_kernel(IndexArgs A) {
  const long b = (long)blockIdx.x * BOXES_PER_BLOCK + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (b >= A.n_boxes) return;
  int i, j, k;
  box_coords(A, b, i, j, k);
  const int rmax = max(max(max(i, A.dims[0] - 1 - i), max(j, A.dims[1] - 1 - j)),
                       max(k, A.dims[2] - 1 - k));
  long top[KSDF_MAX_K];
  for (int t = 0; t < KSDF_MAX_K; ++t) top[t] = LONG_MAX;
  long dk = LONG_MAX;
  for (int r = 0; r <= rmax; ++r) {
    const int cnt = r == 0 ? 1 : 24 * r * r + 2;
    for (int e = lane; e < cnt; e += 64) {
      int dx, dy, dz;
      shell_key(r, e, dx, dy, dz);
      const int x = i + dx, y = j + dy, z = k + dz;
      if (x < 0 || x >= A.dims[0] || y < 0 || y >= A.dims[1] || z < 0 || z >= A.dims[2]) continue;
      if (A.kmap[((long)x * A.dims[1] + y) * A.dims[2] + z] < 0) continue;
      const long far2 = far_units(abs(dx)) + far_units(abs(dy)) + far_units(abs(dz));
      // insert into the sorted private top-K
      if (far2 < top[A.k - 1]) {
        int t = A.k - 1;
        while (t > 0 && top[t - 1] > far2) {
          top[t] = top[t - 1];
          --t;
        }
        top[t] = far2;
      }
    }
    // K rounds of the wave-wide minimum of the private heads: the K-th smallest so far
    int head = 0;
    long kth = LONG_MAX;
    for (int q = 0; q < A.k; ++q) {
      const long mine = head < A.k ? top[head] : LONG_MAX;
      kth = wmin_long(mine);
      if (kth == LONG_MAX) break;
      const unsigned long long who = __ballot(mine == kth);
      if (lane == __ffsll((long long)who) - 1) ++head;
    }
    dk = kth;
    if (kth <= far_units(r + 1) + 2) break;   // no later shell can come nearer
  }
  // rounding margin of the query's FP32 distances: relative, and absolute in
  // proportion to the distance (the coordinates' magnitude is folded into margin_abs)
  long bound = LONG_MAX;
  if (dk < LONG_MAX)
    bound = dk + dk / 65536 + (long)(sqrtf((float)dk) * A.margin_abs);
  int count = 0;
  if (bound < LONG_MAX)
    scan_cube(A, i, j, k, bound, [&](int, bool in) { count += __popcll(__ballot(in)); });
  if (lane == 0) {
    A.bound[b] = bound;
    A.counts[b] = count;
  }
}

__global__ void __launch_bounds__(IDX_THREADS) index_fill_kernel(IndexArgs A) {
  const long b = (long)blockIdx.x * BOXES_PER_BLOCK + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (b >= A.n_boxes) return;
  int i, j, k;
  box_coords(A, b, i, j, k);
  const long bound = A.bound[b];
  if (bound == LONG_MAX) return;
  int pos = A.off[b];
  scan_cube(A, i, j, k, bound, [&](int c, bool in) {
    const unsigned long long bal = __ballot(in);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (in) A.list[pos + before] = c;
    pos += __popcll(bal);
  });
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
  A.kmap = X.kmap;
  A.k = std::min(m->k_fuse, m->n_cells);
  for (int d = 0; d < 3; ++d) A.dims[d] = X.dims[d];
  A.n_boxes = X.n_boxes;
  // A query's squared distance carries rounding of about 2 |x| d 2^-24 per operation,
  // with |x| the coordinates' magnitude and d the distance (sqrt(bound) h / 2); in
  // (h/2)^2 units that is 8 sqrt(bound) (|x| / h) 2^-24 per operation.  The margin
  // takes 2^-16 per sqrt(unit) per box of magnitude, far above that.
  double mag = 0;
  for (int d = 0; d < 3; ++d)
    mag = std::max(mag, std::fabs(m->origin[d]) / m->h + std::max(std::abs(X.lo[d]),
                                                                   std::abs(X.lo[d] + X.dims[d])));
  A.margin_abs = (float)(mag * std::ldexp(1.0, -16));
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
  // the dense map from lattice key to cell id (keys lie inside the lattice, which pads
  // the occupied keys by two boxes)
  std::vector<int> kmap(n_boxes, -1);
  for (int c = 0; c < m->n_cells; ++c) {
    const long x = m->h_keys[3L * c] - X.lo[0], y = m->h_keys[3L * c + 1] - X.lo[1],
               z = m->h_keys[3L * c + 2] - X.lo[2];
    kmap[(x * X.dims[1] + y) * X.dims[2] + z] = c;
  }
  KSDF_HIP_TRY(hipMemcpyAsync(X.kmap, kmap.data(), n_boxes * sizeof(int), hipMemcpyHostToDevice, s));
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
    const long bx = b / ((long)X.dims[1] * X.dims[2]), by = (b / X.dims[2]) % X.dims[1],
               bz = b % X.dims[2];
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
