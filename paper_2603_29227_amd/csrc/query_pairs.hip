// Pair form of the FP32 query's pass 1 (a launch choice of the two-kernel query).
//
// The wave-shared walk of pass 1 evaluates every cell in the union of its 64 lanes'
// candidates for all 64 lanes at once, so with K = 8 candidates per query and a union
// of 15-25 cells per wave most of the issued work is masked off.  Here each (query,
// candidate cell) pair is evaluated exactly once, with the pairs grouped by cell so
// that a wave's lanes share one cell (its samples through scalar loads) and are all
// active:
//   1. candidates: the K nearest cells of every (bucketed) query, stored, and the
//      pairs counted per cell;
//   2. an exclusive scan of the counts, then the pairs (sq * KM + r) scattered into
//      per-cell ranges;
//   3. evaluation of u^2, its error bound and its scaling reference per pair, in the
//      same arithmetic as the wave-shared walk;
//   4. per query, the min-fusion with FP64 re-evaluation of uncertain cells,
//      writing the same record as pass 1 for the regrouping and pass 2.
// Every candidate is evaluated (no lower-bound pruning), as in the method's
// definition of the min-fusion.
#include "query_dev.h"

namespace ksdf {
namespace {

constexpr int PT = 256;

template <int KM>
__global__ void __launch_bounds__(PT) pair_cand_kernel(FastArgs A, int* cand, int* pcount) {
  const long sq = (long)blockIdx.x * PT + threadIdx.x;
  const bool active = sq < A.Q;
  const long qi = active ? A.perm[sq] : 0;
  const float qx = A.pts[3 * qi], qy = A.pts[3 * qi + 1], qz = A.pts[3 * qi + 2];
  int cid[KM];
  int n = 0;
  bool outside = false;
  query_candidates<KM>(A, active, qx, qy, qz, cid, n, outside);
#pragma unroll
  for (int r = 0; r < KM; ++r) {
    const bool v = active && r < n;
    if (active) cand[sq * KM + r] = v ? cid[r] : -1;
    wave_count(pcount, v ? cid[r] : 0, v);
  }
}

template <int KM>
__global__ void __launch_bounds__(PT) pair_scatter_kernel(long Q, const int* cand, int* pcursor,
                                                           int* pairs) {
  const long sq = (long)blockIdx.x * PT + threadIdx.x;
  const bool active = sq < Q;
#pragma unroll
  for (int r = 0; r < KM; ++r) {
    const int c = active ? cand[sq * KM + r] : -1;
    const bool v = c >= 0;
    const int pos = wave_slot(pcursor, v ? c : 0, v);
    if (v) pairs[pos] = (int)(sq * KM + r);
  }
}

// ptotal: the number of pairs (the exclusive scan's entry past the last cell)
template <int KM>
__global__ void __launch_bounds__(PT) pair_eval_kernel(FastArgs A, const int* pairs, const int* cand,
                                                        const int* ptotal, float4* res) {
  const long t = (long)blockIdx.x * PT + threadIdx.x;
  const long total = uniform(*ptotal);
  const bool active = t < total;
  const int p = active ? pairs[t] : 0;
  const int c = active ? cand[p] : -1;
  const long qi = active ? A.perm[p / KM] : 0;
  const float qx = A.pts[3 * qi], qy = A.pts[3 * qi + 1], qz = A.pts[3 * qi + 2];
  float u2 = INFINITY, del = 0.f, d2ref = 0.f;
  bool todo = active;
  // the distinct cells of the wave's pairs (one in almost every wave)
  while (true) {
    unsigned key = todo ? (unsigned)c : 0xffffffffu;
    key = (unsigned)uniform((int)wave_min_u32(key));
    if (key == 0xffffffffu) break;
    const int cc = (int)key;
    const bool mine = todo && c == cc;
    const int b = uniform(A.offsets[cc]);
    const int m = uniform(A.offsets[cc + 1]) - b;
    const float4 ctr = A.centre[cc];
    const float* bx = A.box + 8L * cc;
    const float lx = qx - ctr.x, ly = qy - ctr.y, lz = qz - ctr.z;
    float r2 = aabb_d2(bx, lx, ly, lz);
    float uu, dd;
    cell_u2_wave(A, b, m, lx, ly, lz, mine, r2, uu, dd);
    if (mine) {
      u2 = uu;
      del = dd;
      d2ref = r2;
      todo = false;
    }
  }
  if (active) res[p] = make_float4(u2, del, d2ref, 0.f);
}

template <int KM>
__global__ void __launch_bounds__(PT) pair_fuse_kernel(FastArgs A, const int* cand, const float4* res,
                                                        P1Rec* rec, int* count) {
  const long sq = (long)blockIdx.x * PT + threadIdx.x;
  const bool active = sq < A.Q;
  const long qi = active ? A.perm[sq] : 0;
  const float qx = A.pts[3 * qi], qy = A.pts[3 * qi + 1], qz = A.pts[3 * qi + 2];
  int subkey;
  const bool outside = box_key(A, qx, qy, qz, &subkey) < 0;
  int cid[KM];
  float cu2[KM], cdl[KM], cref[KM];
  int n = 0;
#pragma unroll
  for (int r = 0; r < KM; ++r) {
    const int c = active ? cand[sq * KM + r] : -1;
    cid[r] = c >= 0 ? c : 0x7fffffff;
    cu2[r] = INFINITY;
    cdl[r] = 0.f;
    cref[r] = 0.f;
    if (c >= 0) {
      const float4 v = res[sq * KM + r];
      cu2[r] = v.x;
      cdl[r] = v.y;
      cref[r] = v.z;
      n = r + 1;
    }
  }
  float best = INFINITY;
  const int bc = resolve_min<KM>(A, active, qx, qy, qz, cid, n, cu2, cdl, best);
  float bref = 0.f;
#pragma unroll
  for (int r = 0; r < KM; ++r)
    if (r < n && cid[r] == bc) bref = cref[r];
  Pass1 o;
  o.qx = qx;
  o.qy = qy;
  o.qz = qz;
  o.best = best;
  o.qi = (int)qi;
  o.bc = bc;
  o.bref = bref;
  o.flags = (outside ? 1 : 0) | (active ? 2 : 0);
  if (active) rec[sq] = pack_p1(o);
  wave_count(count, bc < 0 ? A.n_cells : (A.p2rank ? A.p2rank[bc] : bc), active);
}

int km_of(const ksdf_model* m) { return m->k_fuse <= 8 ? 8 : 16; }

}  // namespace

bool query_pairs_usable(const ksdf_model* m, long Q) {
  const long nc = (long)m->n_cells + 1;
  return m->kernel == KSDF_KERNEL_RBF && Q * km_of(m) < (1L << 31) &&
         (nc + SCAN_TILE - 1) / SCAN_TILE <= (long)SCAN_TILE;
}

size_t query_pairs_workspace_bytes(const ksdf_model* m, long Q) {
  const long np = Q * km_of(m);
  const long nc = (long)m->n_cells + 1;
  const long tiles = (nc + SCAN_TILE - 1) / SCAN_TILE;
  return 2 * align256(np * sizeof(int)) + align256(np * sizeof(float4)) +
         2 * align256(nc * sizeof(int)) + align256(tiles * sizeof(int));
}

void launch_pass1_pairs(const ksdf_model* m, const FastArgs& A, P1Rec* rec, int* count, void* ws,
                        hipStream_t s) {
  const int KM = km_of(m);
  const long np = A.Q * KM;
  const long nc = (long)m->n_cells + 1;
  const long tiles = (nc + SCAN_TILE - 1) / SCAN_TILE;
  char* w = static_cast<char*>(ws);
  int* cand = reinterpret_cast<int*>(w);
  w += align256(np * sizeof(int));
  int* pairs = reinterpret_cast<int*>(w);
  w += align256(np * sizeof(int));
  float4* res = reinterpret_cast<float4*>(w);
  w += align256(np * sizeof(float4));
  int* pcount = reinterpret_cast<int*>(w);
  w += align256(nc * sizeof(int));
  int* pcursor = reinterpret_cast<int*>(w);
  w += align256(nc * sizeof(int));
  int* ptsum = reinterpret_cast<int*>(w);
  const unsigned gq = (unsigned)((A.Q + PT - 1) / PT);
  const unsigned gp = (unsigned)((np + PT - 1) / PT);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, pcount, nc, 0);
  if (KM == 8) hipLaunchKernelGGL((pair_cand_kernel<8>), dim3(gq), dim3(PT), 0, s, A, cand, pcount);
  else hipLaunchKernelGGL((pair_cand_kernel<16>), dim3(gq), dim3(PT), 0, s, A, cand, pcount);
  hipLaunchKernelGGL(scan_tiles_kernel, dim3((unsigned)tiles), dim3(SCAN_T), 0, s, pcount, nc, ptsum);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(SCAN_T), 0, s, ptsum, (int)tiles);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)tiles), dim3(SCAN_T), 0, s, pcount, nc, ptsum,
                     pcursor);
  // the scan's entry n_cells (no pair has that key) stays the total through the scatter
  const int* ptotal = pcursor + m->n_cells;
  if (KM == 8) {
    hipLaunchKernelGGL((pair_scatter_kernel<8>), dim3(gq), dim3(PT), 0, s, A.Q, cand, pcursor, pairs);
    hipLaunchKernelGGL((pair_eval_kernel<8>), dim3(gp), dim3(PT), 0, s, A, pairs, cand, ptotal, res);
    hipLaunchKernelGGL((pair_fuse_kernel<8>), dim3(gq), dim3(PT), 0, s, A, cand, res, rec, count);
  } else {
    hipLaunchKernelGGL((pair_scatter_kernel<16>), dim3(gq), dim3(PT), 0, s, A.Q, cand, pcursor, pairs);
    hipLaunchKernelGGL((pair_eval_kernel<16>), dim3(gp), dim3(PT), 0, s, A, pairs, cand, ptotal, res);
    hipLaunchKernelGGL((pair_fuse_kernel<16>), dim3(gq), dim3(PT), 0, s, A, cand, res, rec, count);
  }
}

}  // namespace ksdf
