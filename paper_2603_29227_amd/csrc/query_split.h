// Two-kernel form of the FP32 query (a launch choice with the same outputs as the
// one-kernel form of query_fast.hip).
//
// Pass 1 (candidates, min-fusion) writes one 16-byte record per query in wave order and
// counts the queries of each argmin cell; the records are regrouped by argmin cell;
// pass 2 then meets one or two argmin cells per wave instead of the two to three of
// a spatial bucket, so the per-cell work (gradient, GP variance by forward
// substitution, softmin variance) is not repeated for lanes that idle.
//
// The kernels are instantiated per block size and cell mode in
// query_split{64,256}_{wave,lane}.hip, which compile in parallel.
#pragma once

#include "query_dev.h"

namespace ksdf {
namespace {

// Workgroups go to the chip's 8 XCDs (each with its own L2) in turn: workgroup i runs
// on XCD i mod 8.  Both passes read the cells of neighbouring workgroups (a spatial
// bucket, or one argmin cell's run of records), so each XCD is given one contiguous
// range of the logical workgroups instead: a cell's samples and inverse then fill one
// L2, not eight.  The map is a bijection of [0, n); the results do not depend on it.
constexpr int N_XCD = 8;
__device__ __forceinline__ long xcd_block(long n) {
  const long i = blockIdx.x, q = n / N_XCD, r = n % N_XCD;
  const long x = i % N_XCD, k = i / N_XCD;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

template <int KM, int NT, bool LANE, bool MAT = false>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(KM == 8 ? 5 : 1)))
query_p1_kernel(FastArgs A, P1Rec* rec, int* count) {
  const long sq = xcd_block(gridDim.x) * NT + threadIdx.x;
  const Pass1 r = query_pass1<KM, LANE, MAT>(A, sq);
  const bool active = (r.flags & 2) != 0;
  if (active) rec[sq] = pack_p1(r);
  wave_count(count, r.bc < 0 ? A.n_cells : (A.p2rank ? A.p2rank[r.bc] : r.bc), active);
}

__global__ void __launch_bounds__(256) query_regroup_kernel(const P1Rec* rec, long Q, int n_cells,
                                                            const int* p2rank, int* cursor,
                                                            P1Rec* rec2) {
  const long sq = (long)blockIdx.x * 256 + threadIdx.x;
  const bool active = sq < Q;
  P1Rec r{};
  if (active) r = rec[sq];
  const int bc = p1rec_cell(r);
  const int pos = wave_slot(cursor, bc < 0 ? n_cells : (p2rank ? p2rank[bc] : bc), active);
  if (active) rec2[pos] = r;
}

// split_bin >= 0: the records are grouped by A.p2rank and the launch takes those of
// the cells of rank < split_bin (side 0) or the rest (side 1); their boundary is the
// first record of bin split_bin (its cursor, advanced by the regroup, less its count)
template <int MB, int NT, bool LANE, bool MF = false, bool MAT = false>
__global__ void __launch_bounds__(NT) query_p2_kernel(FastArgs A, const P1Rec* rec2,
                                                      const int* cursor, const int* count,
                                                      int split_bin, int side) {
  long lo = 0, hi = A.Q;
  if (split_bin >= 0) {
    const long S = (long)cursor[split_bin] - count[split_bin];
    if (side == 0) hi = S;
    else lo = S;
  }
  // the blocks of this launch's side [lo, hi) are spread over the 8 XCDs, each XCD one
  // contiguous range of them (as xcd_block does for a whole launch); the launch has a
  // block for every query, rounded up to a multiple of 8, so the blocks past the
  // side's count leave at once
  const long base = lo / NT * NT;
  const long nb = (hi - base + NT - 1) / NT;
  const long per = (nb + N_XCD - 1) / N_XCD;
  const long bx = (long)blockIdx.x % N_XCD, bk = (long)blockIdx.x / N_XCD;
  if (bk >= per || bx * per + bk >= nb) return;   // uniform over the block
  const long sq = base + (bx * per + bk) * NT + threadIdx.x;
  if (split_bin >= 0) {
    const long w0 = sq - (threadIdx.x & 63);
    if (w0 + 64 <= lo || w0 >= hi) return;   // the whole wave is on the other side
  }
  Pass1 r{};
  r.bc = -1;
  if (sq >= lo && sq < hi) {
    const P1Rec o = rec2[sq];
    r.qi = o.qi;
    r.bc = p1rec_cell(o);
    r.flags = (int)(o.cf >> P1REC_CELL_BITS);
    r.best = o.best;
    r.bref = o.bref;
    r.qx = A.pts[3L * o.qi];
    r.qy = A.pts[3L * o.qi + 1];
    r.qz = A.pts[3L * o.qi + 2];
  }
  query_finish_t<MB, LANE, MF, MAT>(A, r);
}

template <int NT, bool LANE>
void launch_split_nt(const ksdf_model* m, const FastArgs& A, P1Rec* rec, P1Rec* rec2, int* count,
                     int* cursor, int* tsum, void* pws, hipStream_t s) {
  const unsigned g = (unsigned)((A.Q + NT - 1) / NT);
  const unsigned g2 = (g + N_XCD - 1) / N_XCD * N_XCD;   // pass 2: whole rounds of the XCDs
  const long nc = (long)m->n_cells + 1;
  const long tiles = (nc + SCAN_TILE - 1) / SCAN_TILE;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, count, nc, 0);
  if (pws) launch_pass1_pairs(m, A, rec, count, pws, s);
  else if (A.matern && m->k_fuse <= 8)
    hipLaunchKernelGGL((query_p1_kernel<8, NT, LANE, true>), dim3(g), dim3(NT), 0, s, A, rec, count);
  else if (A.matern)
    hipLaunchKernelGGL((query_p1_kernel<16, NT, LANE, true>), dim3(g), dim3(NT), 0, s, A, rec, count);
  else if (m->k_fuse <= 8) hipLaunchKernelGGL((query_p1_kernel<8, NT, LANE>), dim3(g), dim3(NT), 0, s, A, rec, count);
  else hipLaunchKernelGGL((query_p1_kernel<16, NT, LANE>), dim3(g), dim3(NT), 0, s, A, rec, count);
  hipLaunchKernelGGL(scan_tiles_kernel, dim3((unsigned)tiles), dim3(SCAN_T), 0, s, count, nc, tsum);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(SCAN_T), 0, s, tsum, (int)tiles);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)tiles), dim3(SCAN_T), 0, s, count, nc, tsum, cursor);
  hipLaunchKernelGGL(query_regroup_kernel, dim3((unsigned)((A.Q + 255) / 256)), dim3(256), 0, s, rec,
                     A.Q, m->n_cells, A.p2rank, cursor, rec2);
  if constexpr (!LANE) {
    if (m->tuning.query_mfma && m->Linv32 && m->max_m <= 64) {
      if (!m->linv_ok) launch_linv(m, s);
      hipLaunchKernelGGL((query_p2_kernel<64, NT, false, true>), dim3(g2), dim3(NT), 0, s, A, rec2,
                         cursor, count, -1, 0);
      return;
    }
  }
  // the kernel function picks the pass-2 instantiation (Matern models carry u, not u^2);
  // with cells of more than 64 samples, the records of the cells of up to 64 run in the
  // launch sized for 64 (fewer registers, more waves per SIMD) and the rest in the one
  // sized for 128
  if (m->max_m <= 64) {
    if (A.matern)
      hipLaunchKernelGGL((query_p2_kernel<64, NT, LANE, false, true>), dim3(g2), dim3(NT), 0, s, A, rec2,
                         cursor, count, -1, 0);
    else
      hipLaunchKernelGGL((query_p2_kernel<64, NT, LANE>), dim3(g2), dim3(NT), 0, s, A, rec2, cursor,
                         count, -1, 0);
    return;
  }
  const int split = m->bucket_start[3];   // ranks of the cells of up to 64 samples
  if (A.matern) {
    hipLaunchKernelGGL((query_p2_kernel<64, NT, LANE, false, true>), dim3(g2), dim3(NT), 0, s, A, rec2,
                       cursor, count, split, 0);
    hipLaunchKernelGGL((query_p2_kernel<128, NT, LANE, false, true>), dim3(g2), dim3(NT), 0, s, A, rec2,
                       cursor, count, split, 1);
  } else {
    hipLaunchKernelGGL((query_p2_kernel<64, NT, LANE>), dim3(g2), dim3(NT), 0, s, A, rec2, cursor, count,
                       split, 0);
    hipLaunchKernelGGL((query_p2_kernel<128, NT, LANE>), dim3(g2), dim3(NT), 0, s, A, rec2, cursor,
                       count, split, 1);
  }
}

}  // namespace
}  // namespace ksdf
