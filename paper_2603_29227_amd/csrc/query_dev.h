// Device bodies of the FP32 query forward, shared by the query kernel and the
// persistent fused fit+query kernel.  See query_fast.hip for the method.
#pragma once

#include <cmath>

#include "ff.h"
#include "wave_ops.h"
#include "ksdf_internal.h"

namespace ksdf {

// Arguments of the FP32 query kernels (shared by the translation units that launch
// them, hence outside the file-local namespace).
struct FastArgs {
  const float* pts;
  long Q;
  const int8_t* sign;
  float* mean;
  float* grad;
  float* var;
  float* var_f;
  float* grad_var;
  int* argmin;
  uint8_t* qst;
  const int* perm;
  // models with cells of more than 64 samples: the split query groups its records by
  // this rank (cells of up to 64 samples first) so that its second kernel runs in two
  // launches sized for 64 and 128 samples; null otherwise (records grouped by cell id)
  const int* p2rank;
  int n_cells;
  int k;
  const int* __restrict__ offsets;
  const long* __restrict__ loff;
  const float4* __restrict__ ps;    // (px, py, pz, a) cell-local
  const float4* __restrict__ plo;   // float-float low parts of (px, py, pz, a)
  const float* __restrict__ sv;
  const float* __restrict__ L;
  const float* __restrict__ Linv;   // [n,64,64] dense L^{-1} (column-major) or null
  const float4* __restrict__ centre;
  const float* __restrict__ box;    // [n,8]: lo xyz, A+, hi xyz, pad
  float origin[3];
  float inv_h;
  int sub;           // sub-boxes per box edge for bucketing (1, 2 or 4)
  int lo[3];
  int dims[3];
  long n_boxes;
  const int* __restrict__ box_off;
  const int* __restrict__ box_rank;
  const int* __restrict__ box_list;
  float c2;          // log2(e) / (2 l^2)
  float two_l2;      // 2 l^2
  float alpha_l2e;   // alpha * log2(e)
  float alpha;
  float inv2l2_ff[2];
  float far2;         // |x - centre|^2 beyond which pass 2 takes the far-field exponent
  float two_l2_ff[2];   // 2 l^2 as a float pair (re-evaluation of uncertain cells)
  // Matern 3/2 models (Table I): k(r) = (1 + c r) e^{-c r}, c = sqrt(3) / l.  Then the
  // per-cell value of pass 1 and the record's `best` are u itself (App. D inverts
  // (1 + c u) e^{-c u} ~ f through the exponential: u = d - ln f' / c), not u^2.
  int matern;
  float mc;            // c
  float mc_l2e;        // c log2(e)
  float mc_ff[2];      // c and 1 / c as float pairs (re-evaluation)
  float inv_mc_ff[2];
};

// What the min-fusion leaves for the argmin cell's outputs: the query, its argmin
// cell (-1: none valid), the minimum u^2 and the scaling reference used for that
// cell (P1Rec below is its stored form).
struct Pass1 {
  float qx, qy, qz, best;
  int qi, bc;
  float bref;
  int flags;   // bit 0: query outside the candidate index; bit 1: active lane;
               // bit 2 (PASS1_FIT_TIMEOUT): read cells whose fit may be unreleased
};
constexpr int PASS1_FIT_TIMEOUT = 4;

// The 16-byte form of a Pass1 that the split query stores between its kernels: the
// query index, the argmin cell + 1 with the flags in the top four bits, the minimum
// and the scaling reference.  The second kernel reads the query point again from the
// caller's points (the same FP32 values the first kernel used).
struct alignas(16) P1Rec {
  int qi;
  unsigned cf;
  float best;
  float bref;
};
constexpr int P1REC_CELL_BITS = 28;   // n_cells + 1 < 2^28 (checked at model creation)

__device__ __forceinline__ P1Rec pack_p1(const Pass1& r) {
  P1Rec o;
  o.qi = r.qi;
  o.cf = (unsigned)(r.bc + 1) | ((unsigned)r.flags << P1REC_CELL_BITS);
  o.best = r.best;
  o.bref = r.bref;
  return o;
}
__device__ __forceinline__ int p1rec_cell(const P1Rec& o) {
  return (int)(o.cf & ((1u << P1REC_CELL_BITS) - 1u)) - 1;
}

// two-kernel query launches (query_split{64,256}_{wave,lane}.hip)
void launch_query_split_64_wave(const ksdf_model* m, const FastArgs& A, P1Rec* rec, P1Rec* rec2,
                               int* count, int* cursor, int* tsum, void* pws, hipStream_t s);
void launch_query_split_64_lane(const ksdf_model* m, const FastArgs& A, P1Rec* rec, P1Rec* rec2,
                               int* count, int* cursor, int* tsum, void* pws, hipStream_t s);
void launch_query_split_256_wave(const ksdf_model* m, const FastArgs& A, P1Rec* rec, P1Rec* rec2,
                               int* count, int* cursor, int* tsum, void* pws, hipStream_t s);
void launch_query_split_256_lane(const ksdf_model* m, const FastArgs& A, P1Rec* rec, P1Rec* rec2,
                               int* count, int* cursor, int* tsum, void* pws, hipStream_t s);
// pair form of pass 1 (query_pairs.hip): usable for Q queries, its workspace, launch
bool query_pairs_usable(const ksdf_model* m, long Q);
size_t query_pairs_workspace_bytes(const ksdf_model* m, long Q);
void launch_pass1_pairs(const ksdf_model* m, const FastArgs& A, P1Rec* rec, int* count, void* ws,
                        hipStream_t s);

namespace {


constexpr int FQ = 256;            // threads per block (4 independent waves)
constexpr float LOG2E = 1.4426950408889634f;
constexpr float LN2 = 0.6931471805599453f;
constexpr float EPS32 = 5.9604645e-08f;



__device__ __forceinline__ unsigned wave_min_u32(unsigned v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, (unsigned)__shfl_xor((int)v, o, 64));
  return v;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ float cand_d2(float qx, float qy, float qz, float4 c) {
  const float dx = __fsub_rn(qx, c.x), dy = __fsub_rn(qy, c.y), dz = __fsub_rn(qz, c.z);
  float t = __fmul_rn(dx, dx);
  t = __fmaf_rn(dy, dy, t);
  return __fmaf_rn(dz, dz, t);
}

// box key of a point in the candidate index (-1 outside) and the Morton index of its
// sub-box when each box is split into sub^3 sub-boxes (sub = 1, 2 or 4)
__device__ __forceinline__ long box_key(const FastArgs& A, float qx, float qy, float qz, int* subkey) {
  const float fx = (qx - A.origin[0]) * A.inv_h, fy = (qy - A.origin[1]) * A.inv_h,
              fz = (qz - A.origin[2]) * A.inv_h;
  const float gx = floorf(fx), gy = floorf(fy), gz = floorf(fz);
  const long kx = (long)gx - A.lo[0], ky = (long)gy - A.lo[1], kz = (long)gz - A.lo[2];
  const int sx = min((int)((fx - gx) * A.sub), A.sub - 1);
  const int sy = min((int)((fy - gy) * A.sub), A.sub - 1);
  const int sz = min((int)((fz - gz) * A.sub), A.sub - 1);
  int mk = 0;
#pragma unroll
  for (int bit = 0; bit < 2; ++bit)
    mk |= (((sx >> bit) & 1) << (3 * bit + 2)) | (((sy >> bit) & 1) << (3 * bit + 1)) |
          (((sz >> bit) & 1) << (3 * bit));
  *subkey = mk;
  if (A.n_boxes <= 0 || kx < 0 || kx >= A.dims[0] || ky < 0 || ky >= A.dims[1] || kz < 0 ||
      kz >= A.dims[2])
    return -1;
  return (kx * A.dims[1] + ky) * A.dims[2] + kz;
}

// ---------------------------------------------------------------------------
// Float-float re-evaluation of one cell's u^2 (rare path), by the whole wave
// ---------------------------------------------------------------------------
// Coordinates and weights come from the float-float store (hi + lo), the differences
// to the query are exact float-float sums, the scaling reference is the nearest
// sample (its float-float z^2), and the kernel values and the log come from
// ff_exp_neg_fast / ff_log (about 2e-12 relative), so that f' carries an error of a
// few parts in 1e12 of sum |a_i e_i| instead of the FP32 pass's 1e-7.  Every lane of
// the wave calls it with the same cell and query; lane l takes samples l, l + 64, ...
// and the nearest-sample minimum and the sum of f' are wave reductions (float-float
// addition is commutative, so every lane ends with the same value).
__device__ __forceinline__ float shfl_xor_f(float v, int o) { return __shfl_xor(v, o, 64); }

__device__ float cell_u2_ff_wave(const FastArgs& A, int c, float qx, float qy, float qz) {
  constexpr int SPL = (KSDF_MAX_M + 63) / 64;
  const int lane = threadIdx.x & 63;
  const int b = A.offsets[c], m = A.offsets[c + 1] - b;
  const float4 ctr = A.centre[c];
  const ff lx = ff_two_sum(qx, -ctr.x), ly = ff_two_sum(qy, -ctr.y), lz = ff_two_sum(qz, -ctr.z);
  ff z2[SPL];
  ff d2{INFINITY, 0.f};
#pragma unroll
  for (int k = 0; k < SPL; ++k) {
    const int i = lane + 64 * k;
    z2[k] = ff{INFINITY, 0.f};
    if (i < m) {
      const float4 p = A.ps[b + i], pl = A.plo[b + i];
      const ff dx = ff_add(lx, ff{-p.x, -pl.x});
      const ff dy = ff_add(ly, ff{-p.y, -pl.y});
      const ff dz = ff_add(lz, ff{-p.z, -pl.z});
      z2[k] = ff_add(ff_add(ff_mul(dx, dx), ff_mul(dy, dy)), ff_mul(dz, dz));
      if (z2[k].hi < d2.hi || (z2[k].hi == d2.hi && z2[k].lo < d2.lo)) d2 = z2[k];
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const ff t{shfl_xor_f(d2.hi, o), shfl_xor_f(d2.lo, o)};
    if (t.hi < d2.hi || (t.hi == d2.hi && t.lo < d2.lo)) d2 = t;
  }
  const ff inv{A.inv2l2_ff[0], A.inv2l2_ff[1]};
  ff f{0.f, 0.f};
#pragma unroll
  for (int k = 0; k < SPL; ++k) {
    const int i = lane + 64 * k;
    if (i < m) {
      const float aw = A.ps[b + i].w, awl = A.plo[b + i].w;
      const ff t = ff_mul(ff_add(z2[k], ff_neg(d2)), inv);
      f = ff_add(f, ff_mul(ff{aw, awl}, ff_exp_neg_fast(t)));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) f = ff_add(f, ff{shfl_xor_f(f.hi, o), shfl_xor_f(f.lo, o)});
  if (!(f.hi > 0.f)) return INFINITY;
  const ff u2 = ff_add(d2, ff_neg(ff_mul(ff{A.two_l2_ff[0], A.two_l2_ff[1]}, ff_log(f))));
  return u2.hi + u2.lo;
}

// The Matern 3/2 counterpart: u = d - ln f' / c with f' = sum a_i (1 + c z_i)
// e^{-c (z_i - d)} and d the nearest sample's distance, every step in float-float
// (square roots by one Newton step on the exact residual).
__device__ float cell_u_matern_ff_wave(const FastArgs& A, int c, float qx, float qy, float qz) {
  constexpr int SPL = (KSDF_MAX_M + 63) / 64;
  const int lane = threadIdx.x & 63;
  const int b = A.offsets[c], m = A.offsets[c + 1] - b;
  const float4 ctr = A.centre[c];
  const ff lx = ff_two_sum(qx, -ctr.x), ly = ff_two_sum(qy, -ctr.y), lz = ff_two_sum(qz, -ctr.z);
  ff z2[SPL];
  ff d2{INFINITY, 0.f};
#pragma unroll
  for (int k = 0; k < SPL; ++k) {
    const int i = lane + 64 * k;
    z2[k] = ff{INFINITY, 0.f};
    if (i < m) {
      const float4 p = A.ps[b + i], pl = A.plo[b + i];
      z2[k] = ff_norm2_lean(ff_sub_lean(lx.hi, lx.lo, p.x, pl.x), ff_sub_lean(ly.hi, ly.lo, p.y, pl.y),
                            ff_sub_lean(lz.hi, lz.lo, p.z, pl.z));
      if (z2[k].hi < d2.hi || (z2[k].hi == d2.hi && z2[k].lo < d2.lo)) d2 = z2[k];
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const ff t{shfl_xor_f(d2.hi, o), shfl_xor_f(d2.lo, o)};
    if (t.hi < d2.hi || (t.hi == d2.hi && t.lo < d2.lo)) d2 = t;
  }
  const ff cc{A.mc_ff[0], A.mc_ff[1]};
  const ff d = ff_sqrt(d2);
  ff f{0.f, 0.f};
#pragma unroll
  for (int k = 0; k < SPL; ++k) {
    const int i = lane + 64 * k;
    if (i < m) {
      const float aw = A.ps[b + i].w, awl = A.plo[b + i].w;
      const ff z = ff_sqrt(z2[k]);
      const ff t = ff_mul(ff_add(z, ff_neg(d)), cc);
      const ff g = ff_add(ff{1.f, 0.f}, ff_mul(z, cc));
      f = ff_add(f, ff_mul(ff{aw, awl}, ff_mul(g, ff_exp_neg_lean(t))));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) f = ff_add(f, ff{shfl_xor_f(f.hi, o), shfl_xor_f(f.lo, o)});
  if (!(f.hi > 0.f)) return INFINITY;
  const ff u = ff_add(d, ff_neg(ff_mul(ff_log(f), ff{A.inv_mc_ff[0], A.inv_mc_ff[1]})));
  return u.hi + u.lo;
}

// lower bound of the squared distance from local point (x,y,z) to the cell's
// sample bounding box
__device__ __forceinline__ float aabb_d2(const float* bx, float x, float y, float z) {
  const float ex = fmaxf(fmaxf(bx[0] - x, 0.f), x - bx[4]);
  const float ey = fmaxf(fmaxf(bx[1] - y, 0.f), y - bx[5]);
  const float ez = fmaxf(fmaxf(bx[2] - z, 0.f), z - bx[6]);
  return ex * ex + ey * ey + ez * ez;
}

// Error budget on u^2.  The accuracy target is 1e-4 m relative to max(u, 1 m), and
// 2 l^2 * 1e-5 on u^2 near u = 0 where the square root amplifies errors.  The
// per-cell error bound del (a worst-case sum of per-term rounding errors) was
// measured against FP64 on 52k room queries: the actual error never exceeded 0.31
// of it (median 0.02).  A cell is re-evaluated in float-float when 0.35 * del could
// reach half the target, i.e. del > BUDGET_SCALE * target.
constexpr float BUDGET_SCALE = 0.5f / 0.35f;
__device__ __forceinline__ float u2_budget(float u2, float two_l2) {
  const float u = sqrtf(fmaxf(u2, 0.f));
  return BUDGET_SCALE * fmaxf(two_l2 * 1e-5f, 2.f * u * 1e-4f * fmaxf(u, 1.f));
}
// Matern: pass 1 carries u, so the target applies directly
__device__ __forceinline__ float u_budget(float u) {
  return BUDGET_SCALE * 1e-4f * fmaxf(fabsf(u), 1.f);
}

// Sample-chunk size of the wave-uniform loops: one group of scalar loads (8 float4 =
// 32 SGPRs) feeds 8 evaluations, so a wave waits once per 8 samples on the scalar
// cache and the other waves of the SIMD fill that wait.
constexpr int CH = 8;

// packed row index of stream position e (compile-time after unrolling)
__host__ __device__ constexpr int row_of(int e) {
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= e) ++i;
  return i;
}

// v <- L^{-1} v for the first m rows (L packed by rows with reciprocal diagonal),
// streaming the packed factor LC floats at a time (through scalar registers when the
// cell is wave-uniform).  The chunks are generated by template recursion so every
// (row, column) index is a compile-time constant and v stays in registers.
// Accumulates |L^{-1} v|^2 over the first m rows into vv.
template <int E0, int MB, int LC>
__device__ __forceinline__ void fsub_chunk(const float* __restrict__ Lc, int m, float (&v)[MB],
                                           float& vv, float& t) {
  constexpr int NP = MB * (MB + 1) / 2;
  if constexpr (E0 < NP) {
    if (row_of(E0) >= m) return;
    float buf[LC];
#pragma unroll
    for (int q = 0; q < LC; ++q) buf[q] = Lc[E0 + q];
#pragma unroll
    for (int q = 0; q < LC; ++q) {
      const int e = E0 + q;
      if (e < NP) {
        const int i = row_of(e), j = e - i * (i + 1) / 2;
        if (j == 0) t = v[i];
        if (j < i) {
          t = fmaf(-buf[q], v[j], t);
        } else {
          v[i] = t * buf[q];
          if (i < m) vv = fmaf(v[i], v[i], vv);
        }
      }
    }
    fsub_chunk<E0 + LC, MB, LC>(Lc, m, v, vv, t);
  }
}

// LC: factor entries per load group (32 through scalar registers when the cell is
// wave-uniform; fewer when every lane loads its own cell into vector registers)
template <int MB, int LC = 32>
__device__ __forceinline__ float forward_subst(const float* __restrict__ Lc, int m, float (&v)[MB]) {
  float vv = 0.f, t = 0.f;
  fsub_chunk<0, MB, LC>(Lc, m, v, vv, t);
  return vv;
}

__device__ __forceinline__ float readlane_f(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Top-KM of (distance, id) over the list of index box b0, for a wave whose active lanes
// all lie in that box (every lane of the wave calls it; `ref` is an active lane).  Lane
// j loads entry j of each 64-entry chunk of the list; the chunk is sorted across the
// wave (bitonic) by its distance to the query of lane ref, so that every lane meets
// its nearest cells early and later entries rarely enter; the entries then reach all
// lanes by readlane.  They do not arrive in id order, so equal distances are ordered
// by id explicitly, which gives the same top-KM as the scan in id order.
template <int KM>
__device__ __forceinline__ void candidates_shared_box(const FastArgs& A, bool active, float qx,
                                                      float qy, float qz, int b0, int ref,
                                                      float (&cd)[KM], int (&cid)[KM], int& len) {
  const int lane = threadIdx.x & 63;
  const int beg = uniform(A.box_off[b0]), end = uniform(A.box_off[b0 + 1]);
  len = end - beg;
  const float rx = readlane_f(qx, ref), ry = readlane_f(qy, ref), rz = readlane_f(qz, ref);
  for (int t0 = beg; t0 < end; t0 += 64) {
    const int t = t0 + lane;
    const bool have = t < end;
    const int id = have ? A.box_list[t] : 0;
    const float4 ce = A.centre[id];
    float key = have ? cand_d2(rx, ry, rz, ce) : INFINITY;
    int src = lane;
#pragma unroll
    for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
      for (int j = size >> 1; j > 0; j >>= 1) {
        const float ok = __shfl_xor(key, j, 64);
        const int os = __shfl_xor(src, j, 64);
        // ascending blocks keep the smaller pair in the lower lane, descending the larger
        const bool keep_min = ((lane & j) == 0) == ((lane & size) == 0);
        const bool other_less = ok < key || (ok == key && os < src);
        if (other_less == keep_min) {
          key = ok;
          src = os;
        }
      }
    }
    const int cnt = min(64, end - t0);
    for (int e = 0; e < cnt; ++e) {
      const int s = __builtin_amdgcn_readlane(src, e);
      int xi = __builtin_amdgcn_readlane(id, s);
      const float4 c = make_float4(readlane_f(ce.x, s), readlane_f(ce.y, s), readlane_f(ce.z, s), 0.f);
      float x = cand_d2(qx, qy, qz, c);
      if (active && (x < cd[KM - 1] || (x == cd[KM - 1] && xi < cid[KM - 1]))) {
#pragma unroll
        for (int r = 0; r < KM; ++r) {
          if (x < cd[r] || (x == cd[r] && xi < cid[r])) {
            const float tx = cd[r];
            const int ti = cid[r];
            cd[r] = x;
            cid[r] = xi;
            x = tx;
            xi = ti;
          }
        }
      }
    }
  }
}

// K nearest occupied cell centres of the candidate-index box list of (qx,qy,qz), ties
// by id (Sec. IV-B.1): the first n entries of cid, nearest first.  outside: the point
// lies outside the index lattice (then every cell is scanned).  Every lane of the wave
// calls it together.
template <int KM>
__device__ __forceinline__ void query_candidates(const FastArgs& A, bool active, float qx, float qy,
                                                 float qz, int (&cid)[KM], int& n, bool& outside) {
  // sorted top-KM of (distance, id), compared as pairs: an entry displaced by an
  // insertion moves down past equal distances only in id order; the first k entries
  // are the K nearest
  float cd[KM];
#pragma unroll
  for (int r = 0; r < KM; ++r) {
    cd[r] = INFINITY;
    cid[r] = 0x7fffffff;
  }
  int subkey;
  const long bkey = box_key(A, qx, qy, qz, &subkey);
  outside = bkey < 0;
  n = 0;
  const unsigned long long act = __ballot(active);
  if (act) {
    const int ref = __builtin_ctzll(act);
    const int b0 = __builtin_amdgcn_readlane((int)bkey, ref);
    if (b0 >= 0 && !__ballot(active && bkey != b0)) {
      int len;
      candidates_shared_box<KM>(A, active, qx, qy, qz, b0, ref, cd, cid, len);
      n = active ? min(A.k, len) : 0;
      return;
    }
  }
  if (active) {
    int beg = 0, end = A.n_cells;
    if (!outside) {
      beg = A.box_off[bkey];
      end = A.box_off[bkey + 1];
    }
    for (int t0 = beg; t0 < end; t0 += 4) {
      int cc[4];
      float4 ce[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = min(t0 + u, end - 1);
        cc[u] = outside ? t : A.box_list[t];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) ce[u] = A.centre[cc[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool in = t0 + u < end;
        float x = in ? cand_d2(qx, qy, qz, ce[u]) : INFINITY;
        int xi = in ? cc[u] : 0x7fffffff;
        if (x < cd[KM - 1] || (x == cd[KM - 1] && xi < cid[KM - 1])) {
#pragma unroll
          for (int r = 0; r < KM; ++r) {
            if (x < cd[r] || (x == cd[r] && xi < cid[r])) {
              const float tx = cd[r];
              const int ti = cid[r];
              cd[r] = x;
              cid[r] = xi;
              x = tx;
              xi = ti;
            }
          }
        }
      }
    }
    n = min(A.k, end - beg);
  }
}

// One chunk of CH samples of the u^2 sums: f = sum a e, R = sum |a| e, RZ = sum |a| e z^2,
// emax = max e, with e = 2^(c2 (d2ref - z^2)).  With MASK, entries past m belong to the
// next cell (the store is padded): their offsets from this cell's centre can be far
// nearer than d2ref, and exp2 would overflow, so their term is masked, not weighted by 0.
template <bool MASK>
__device__ __forceinline__ void u2_chunk(const float4 (&P)[CH], int i0, int m, float lx, float ly,
                                         float lz, float c2, float c2d, float& f, float& R,
                                         float& RZ, float& emax) {
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    const bool in = !MASK || i0 + j < m;
    const float aw = P[j].w;
    const float dx = lx - P[j].x, dy = ly - P[j].y, dz = lz - P[j].z;
    const float z2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const float e = in ? __builtin_amdgcn_exp2f(fmaf(z2, -c2, c2d)) : 0.f;
    const float ae = fabsf(aw) * e;
    f = fmaf(aw, e, f);
    R += ae;
    RZ = fmaf(ae, z2, RZ);
    emax = fmaxf(emax, e);
  }
}

// u^2 of one cell at the cell-local point (lx,ly,lz) for the lanes with ev set, with
// its rounding-error bound del, against the scaling reference d2ref (in: the sample
// box's lower bound; out: the reference used).  Wave-uniform: every lane of the wave
// calls it for the same cell (b, m), whose samples come through scalar loads.
__device__ __forceinline__ void cell_u2_wave(const FastArgs& A, int b, int m, float lx, float ly,
                                             float lz, bool ev, float& d2ref, float& u2,
                                             float& del) {
  const float c2 = A.c2;
  u2 = INFINITY;
  del = 0.f;
  if (!__ballot(ev)) return;
  float f = 0.f, R = 0.f, RZ = 0.f;
  for (int pass = 0; pass < 2; ++pass) {
    const float c2d = c2 * d2ref;
    float emax = 0.f;
    f = 0.f;
    R = 0.f;
    RZ = 0.f;
    for (int i0 = 0; i0 < m; i0 += CH) {
      float4 P[CH];
#pragma unroll
      for (int j = 0; j < CH; ++j) P[j] = A.ps[b + i0 + j];   // the store is padded
      // only the last chunk of a cell needs the mask (the test is wave-uniform)
      if (i0 + CH <= m) u2_chunk<false>(P, i0, m, lx, ly, lz, c2, c2d, f, R, RZ, emax);
      else u2_chunk<true>(P, i0, m, lx, ly, lz, c2, c2d, f, R, RZ, emax);
    }
    // far from the cell, the nearest sample can lie so much farther than the box's
    // nearest point that every term is tiny against the box reference and the
    // smaller ones underflow (FP32 exponents end at -126): redo once against the
    // nearest sample, which gives its own term 1
    const bool low = ev && !(emax >= 0x1p-24f);
    if (!__ballot(low)) break;
    if (low) {
      float d2 = INFINITY;
      for (int i = 0; i < m; ++i) {
        const float4 p = A.ps[b + i];
        const float dx = lx - p.x, dy = ly - p.y, dz = lz - p.z;
        d2 = fminf(d2, fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
      }
      d2ref = d2;
    }
  }
  if (ev && f > 0.f) {
    u2 = d2ref - A.two_l2 * LN2 * __log2f(f);
    // |d f| <= eps * sum_i |a_i| e_i (2 + (5 ln 2) c2 z_i^2) + summation error
    del = A.two_l2 * EPS32 * (6.f * R + 3.5f * c2 * RZ) / f;
  }
}

// Matern 3/2 pass-1 sums over one chunk: f = sum a g, R = sum |a| g, RZ = sum |a| g z
// with g_i = (1 + c z_i) 2^(c log2(e) (dref - z_i)) and emax the largest exponential
// factor; dref <= every z_i (the sample box's lower bound), so no factor exceeds 1.
template <bool MASK>
__device__ __forceinline__ void um_chunk(const float4 (&P)[CH], int i0, int m, float lx, float ly,
                                         float lz, float mc, float mcl, float dref, float& f,
                                         float& R, float& RZ, float& emax) {
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    const bool in = !MASK || i0 + j < m;
    const float aw = P[j].w;
    const float dx = lx - P[j].x, dy = ly - P[j].y, dz = lz - P[j].z;
    const float z = __builtin_amdgcn_sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
    const float ex = in ? __builtin_amdgcn_exp2f(mcl * (dref - z)) : 0.f;
    const float g = fmaf(mc, z, 1.f) * ex;
    const float ag = fabsf(aw) * g;
    f = fmaf(aw, g, f);
    R += ag;
    RZ = fmaf(ag, z, RZ);
    emax = fmaxf(emax, ex);
  }
}

// u = dref - ln(f') / c of one Matern cell and its rounding-error bound: each term
// carries at most eps (5 + 3 c z_i) relative error (the root, the exponent's argument
// c (dref - z_i), the factor 1 + c z_i, the products) and the sum a few eps of
// sum |terms|, so |d f'| <= eps (8 R + 4 c RZ) and |d u| <= |d f'| / (c f').
// Wave-uniform like cell_u2_wave (same two-pass underflow rule).
__device__ __forceinline__ void cell_u_matern_wave(const FastArgs& A, int b, int m, float lx,
                                                   float ly, float lz, bool ev, float& d2ref,
                                                   float& u, float& del) {
  const float mc = A.mc, mcl = A.mc_l2e;
  u = INFINITY;
  del = 0.f;
  if (!__ballot(ev)) return;
  float f = 0.f, R = 0.f, RZ = 0.f;
  for (int pass = 0; pass < 2; ++pass) {
    const float dref = __builtin_amdgcn_sqrtf(d2ref);
    float emax = 0.f;
    f = 0.f;
    R = 0.f;
    RZ = 0.f;
    for (int i0 = 0; i0 < m; i0 += CH) {
      float4 P[CH];
#pragma unroll
      for (int j = 0; j < CH; ++j) P[j] = A.ps[b + i0 + j];   // the store is padded
      if (i0 + CH <= m) um_chunk<false>(P, i0, m, lx, ly, lz, mc, mcl, dref, f, R, RZ, emax);
      else um_chunk<true>(P, i0, m, lx, ly, lz, mc, mcl, dref, f, R, RZ, emax);
    }
    const bool low = ev && !(emax >= 0x1p-24f);
    if (!__ballot(low)) break;
    if (low) {
      float d2 = INFINITY;
      for (int i = 0; i < m; ++i) {
        const float4 p = A.ps[b + i];
        const float dx = lx - p.x, dy = ly - p.y, dz = lz - p.z;
        d2 = fminf(d2, fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
      }
      d2ref = d2;
    }
  }
  if (ev && f > 0.f) {
    u = __builtin_amdgcn_sqrtf(d2ref) - LN2 * __log2f(f) / mc;
    del = EPS32 * (8.f * R + 4.f * mc * RZ) / (mc * f);
  }
}

// The per-lane (vector-load) form of the same, for the sparse-query walk.
__device__ __forceinline__ void cell_u_matern_lane(const FastArgs& A, int b, int m, float lx,
                                                   float ly, float lz, float& d2ref, float& u,
                                                   float& del) {
  const float mc = A.mc, mcl = A.mc_l2e;
  float f = 0.f, R = 0.f, RZ = 0.f;
  u = INFINITY;
  del = 0.f;
  for (int pass = 0; pass < 2; ++pass) {
    const float dref = __builtin_amdgcn_sqrtf(d2ref);
    float emax = 0.f;
    f = 0.f;
    R = 0.f;
    RZ = 0.f;
    for (int i = 0; i < m; ++i) {
      const float4 P = A.ps[b + i];
      const float dx = lx - P.x, dy = ly - P.y, dz = lz - P.z;
      const float z = __builtin_amdgcn_sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
      const float ex = __builtin_amdgcn_exp2f(mcl * (dref - z));
      const float g = fmaf(mc, z, 1.f) * ex;
      const float ag = fabsf(P.w) * g;
      f = fmaf(P.w, g, f);
      R += ag;
      RZ = fmaf(ag, z, RZ);
      emax = fmaxf(emax, ex);
    }
    if (emax >= 0x1p-24f) break;
    float d2 = INFINITY;
    for (int i = 0; i < m; ++i) {
      const float4 p = A.ps[b + i];
      const float dx = lx - p.x, dy = ly - p.y, dz = lz - p.z;
      d2 = fminf(d2, fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
    }
    d2ref = d2;
  }
  if (f > 0.f) {
    u = __builtin_amdgcn_sqrtf(d2ref) - LN2 * __log2f(f) / mc;
    del = EPS32 * (8.f * R + 4.f * mc * RZ) / (mc * f);
  }
}

// Lower bound of a cell's value from its sample box: RBF u^2 >= d^2 - 2 l^2 ln max(A+, 1)
// (every scaled term is at most a_i); Matern u >= d - ln(max(A+, 1) (1 + c d)) / c
// ((1 + c z) e^{-c (z - d)} decreases in z >= d, so each term is at most a_i (1 + c d)).
__device__ __forceinline__ float cell_lower_bound(const FastArgs& A, float d2box, float apos) {
  if (A.matern) {
    const float d = __builtin_amdgcn_sqrtf(d2box);
    return d - logf(fmaxf(apos, 1.f) * fmaf(A.mc, d, 1.f)) / A.mc;
  }
  return d2box - A.two_l2 * logf(fmaxf(apos, 1.f));
}

// Min-fusion of the candidates' u^2 (ties to the lower id), with float-float
// re-evaluation where FP32 could be off by more than the error budget: the best
// cell's own error may take half of it, and the misordering of the best and a rival
// whose error band overlaps it (at most the sum of their errors) the other half.
// While a condition fails, the cell with the larger error of the failing pair is
// re-evaluated (its error then counts as zero) and the conditions are checked again,
// so near-tied cells of small error are not redone.  Returns the argmin cell (-1:
// none valid); best = its u^2.
template <int KM>
__device__ __forceinline__ int resolve_min(const FastArgs& A, bool active, float qx, float qy,
                                           float qz, const int (&cid)[KM], int n, float (&cu2)[KM],
                                           float (&cdl)[KM], float& best) {
  auto argmin = [&](float& bu, float& bd, int& bs) {
    int c = -1;
    bu = INFINITY;
    bd = 0.f;
    bs = 0;
#pragma unroll
    for (int r = 0; r < KM; ++r)
      if (r < n && (cu2[r] < bu || (cu2[r] == bu && cu2[r] < INFINITY && cid[r] < c))) {
        bu = cu2[r];
        bd = cdl[r];
        c = cid[r];
        bs = r;
      }
    return c;
  };
  // the slot to re-evaluate next (a one-bit mask), or 0 when the budget holds
  auto next = [&](int bc, float bu, float bd, int bs) -> unsigned {
    if (bc < 0) return 0u;
    const float budget = A.matern ? u_budget(bu) : u2_budget(bu, A.two_l2);
    if (bd > budget) return 1u << bs;
    int pick = -1;
    float worst = 0.f;
#pragma unroll
    for (int r = 0; r < KM; ++r)
      if (r != bs && r < n && cu2[r] < INFINITY && cu2[r] - cdl[r] <= bu + bd &&
          cdl[r] + bd > budget) {
        const float e = fmaxf(cdl[r], bd);
        if (e > worst) {
          worst = e;
          pick = cdl[r] >= bd ? r : bs;
        }
      }
    return pick >= 0 ? 1u << pick : 0u;
  };
  float bu = INFINITY, bd = 0.f;
  int bs = 0;
  int bc = active ? argmin(bu, bd, bs) : -1;
  const bool found = bc >= 0;
  unsigned need = active ? next(bc, bu, bd, bs) : 0u;
  // the wave takes the flagged (query, cell) pairs one at a time, lowest lane first
  while (true) {
    const unsigned long long pend = __ballot(need != 0);
    if (!pend) break;
    const int src = __builtin_ctzll(pend);
    const int myr = need ? __builtin_ctz(need) : 0;
    int myc = 0;
#pragma unroll
    for (int r = 0; r < KM; ++r)
      if (r == myr) myc = cid[r];
    const int c = __builtin_amdgcn_readlane(myc, src);
    const int rs = __builtin_amdgcn_readlane(myr, src);
    const float sx = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, qx), src));
    const float sy = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, qy), src));
    const float sz = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, qz), src));
    const float u2 = A.matern ? cell_u_matern_ff_wave(A, c, sx, sy, sz)
                              : cell_u2_ff_wave(A, c, sx, sy, sz);
    if ((int)(threadIdx.x & 63) == src) {
#pragma unroll
      for (int r = 0; r < KM; ++r)
        if (r == rs) {
          cu2[r] = u2;
          cdl[r] = 0.f;
        }
      bc = argmin(bu, bd, bs);
      need = next(bc, bu, bd, bs);
    }
  }
  if (found) best = bu;
  return bc;
}

// Candidates, per-candidate u^2 and the min-fusion for the 64 sorted queries sq ..
// of a wave (lanes pass their own sq); every lane of the wave must call it together
// (wave-uniform loops inside).
template <int KM, bool LANE = false, bool MAT = false>
__device__ __forceinline__ Pass1 query_pass1(const FastArgs& A, long sq) {
  const bool active = sq < A.Q;
  const long qi = active ? A.perm[sq] : 0;
  const float qx = A.pts[3 * qi], qy = A.pts[3 * qi + 1], qz = A.pts[3 * qi + 2];

  // ---- candidates: K nearest centres of the box list (ties by id)
  int cid[KM];
  int n = 0;
  bool outside = false;
  query_candidates<KM>(A, active, qx, qy, qz, cid, n, outside);

  // ---- pass 1: per-candidate u^2 with error bounds, wave-uniform over the union
  float cu2[KM], cdl[KM], cref[KM];
#pragma unroll
  for (int r = 0; r < KM; ++r) {
    cu2[r] = INFINITY;
    cdl[r] = 0.f;
    cref[r] = 0.f;
  }
  float best = INFINITY, best_del = 0.f;
  const float c2 = A.c2;
  if constexpr (!LANE) {
  unsigned pending = active ? ((1u << n) - 1u) : 0u;
  while (true) {
    unsigned key = 0xffffffffu;
    if (pending) {
      const int r0 = __ffs(pending) - 1;
      int c0 = 0;
#pragma unroll
      for (int r = 0; r < KM; ++r)
        if (r == r0) c0 = cid[r];
      key = ((unsigned)r0 << 24) | (unsigned)c0;
    }
    key = (unsigned)uniform((int)wave_min_u32(key));
    if (key == 0xffffffffu) break;
    const int c = (int)(key & 0xffffffu);
    int slot = -1;
#pragma unroll
    for (int r = 0; r < KM; ++r)
      if (((pending >> r) & 1u) && cid[r] == c) slot = r;
    const int b = uniform(A.offsets[c]);
    const int m = uniform(A.offsets[c + 1]) - b;
    const float4 ctr = A.centre[c];
    const float* bx = A.box + 8L * c;
    const float lx = qx - ctr.x, ly = qy - ctr.y, lz = qz - ctr.z;
    float d2ref = aabb_d2(bx, lx, ly, lz);
    const float lb = cell_lower_bound(A, d2ref, bx[3]);
    const bool part = slot >= 0;
    const bool ev = part && !(lb > best + 2.f * best_del + 1e-6f);
    float u2 = INFINITY, del = 0.f;
    if constexpr (MAT) cell_u_matern_wave(A, b, m, lx, ly, lz, ev, d2ref, u2, del);
    else cell_u2_wave(A, b, m, lx, ly, lz, ev, d2ref, u2, del);
    if (part) {
      if (!ev) u2 = INFINITY;   // pruned: provably not the minimum
#pragma unroll
      for (int r = 0; r < KM; ++r)
        if (r == slot) {
          cu2[r] = u2;
          cdl[r] = del;
        }
#pragma unroll
      for (int r = 0; r < KM; ++r)
        if (r == slot) cref[r] = d2ref;
      pending &= ~(1u << slot);
      if (u2 < best) {
        best = u2;
        best_del = del;
      }
    }
  }
  } else {
    // per lane: each lane walks its own candidates, nearest centre first, with its
    // own (vector) loads; for sparse queries, whose waves would share few cells.
    // The same arithmetic in the same order as the wave-uniform walk, so the same
    // results.
#pragma unroll
    for (int r = 0; r < KM; ++r) {
      if (active && r < n) {
        const int c = cid[r];
        const int b = A.offsets[c];
        const int m = A.offsets[c + 1] - b;
        const float4 ctr = A.centre[c];
        const float* bx = A.box + 8L * c;
        const float lx = qx - ctr.x, ly = qy - ctr.y, lz = qz - ctr.z;
        float d2ref = aabb_d2(bx, lx, ly, lz);
        const float lb = cell_lower_bound(A, d2ref, bx[3]);
        float u2 = INFINITY, del = 0.f;
        if constexpr (MAT) {
          if (!(lb > best + 2.f * best_del + 1e-6f)) cell_u_matern_lane(A, b, m, lx, ly, lz, d2ref, u2, del);
        } else if (!(lb > best + 2.f * best_del + 1e-6f)) {
          float f = 0.f, R = 0.f, RZ = 0.f;
          for (int pass = 0; pass < 2; ++pass) {
            const float c2d = c2 * d2ref;
            float emax = 0.f;
            f = 0.f;
            R = 0.f;
            RZ = 0.f;
            for (int i = 0; i < m; ++i) {
              const float4 P = A.ps[b + i];
              const float dx = lx - P.x, dy = ly - P.y, dz = lz - P.z;
              const float z2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
              const float e = __builtin_amdgcn_exp2f(fmaf(z2, -c2, c2d));
              const float ae = fabsf(P.w) * e;
              f = fmaf(P.w, e, f);
              R += ae;
              RZ = fmaf(ae, z2, RZ);
              emax = fmaxf(emax, e);
            }
            if (emax >= 0x1p-24f) break;
            float d2 = INFINITY;
            for (int i = 0; i < m; ++i) {
              const float4 p = A.ps[b + i];
              const float dx = lx - p.x, dy = ly - p.y, dz = lz - p.z;
              d2 = fminf(d2, fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
            }
            d2ref = d2;
          }
          if (f > 0.f) {
            u2 = d2ref - A.two_l2 * LN2 * __log2f(f);
            del = A.two_l2 * EPS32 * (6.f * R + 3.5f * c2 * RZ) / f;
          }
        }
        cu2[r] = u2;
        cdl[r] = del;
        cref[r] = d2ref;
        if (u2 < best) {
          best = u2;
          best_del = del;
        }
      }
    }
  }

  // ---- resolve the minimum; re-evaluate uncertain cells in float-float
  const int bc = resolve_min<KM>(A, active, qx, qy, qz, cid, n, cu2, cdl, best);
  // the argmin cell's scaling reference from pass 1 (box bound, or its nearest sample
  // where the box bound would have underflowed the terms)
  float bref = 0.f;
#pragma unroll
  for (int r = 0; r < KM; ++r)
    if (r < n && cid[r] == bc) bref = cref[r];
  Pass1 r;
  r.qx = qx;
  r.qy = qy;
  r.qz = qz;
  r.best = best;
  r.qi = (int)qi;
  r.bc = bc;
  r.bref = bref;
  r.flags = (outside ? 1 : 0) | (active ? 2 : 0);
  return r;
}

// Variance of the softmin gradient g = sum_i l_i v_i of one cell (App. C): the
// derivative of g with respect to sample i is
//   J_i = alpha w_i v_i^T + (l_i / z_i)(v_i v_i^T - I),  w_i = l_i (v_i - Vs) + s_i (v_i - g),
// with v_i the unit vector from sample i to the query, s the normalised softmin
// weights, l_i = s_i (alpha h - alpha z_i + 1) and Vs = sum s_i v_i.  As |v_i| = 1,
// row k of J_i has squared norm alpha^2 w_ik^2 + (l_i / z_i)^2 (1 - v_ik^2), and
// V[grad_k u] = sum_i sigma_i^2 |row k of J_i|^2.  With t_i = alpha (z_i - zref) and
// the unnormalised weights e^{-t_i}: s_i = e^{-t_i} / S and l_i = s_i (Tb - t_i).
// Two more passes over the cell's samples (the sums Vs and g first); called only
// when the caller asks for the output.
__device__ __forceinline__ float3 grad_var_cell(const FastArgs& A, int b, int m, float lx,
                                                float ly, float lz, float zref, float S,
                                                float Tb) {
  const float invS = 1.f / S;
  float V0 = 0.f, V1 = 0.f, V2 = 0.f, G0 = 0.f, G1 = 0.f, G2 = 0.f;
  for (int i = 0; i < m; ++i) {
    const float4 P = A.ps[b + i];
    const float dx = lx - P.x, dy = ly - P.y, dz = lz - P.z;
    const float z = __builtin_amdgcn_sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
    if (!(z > 0.f)) continue;
    const float s = __builtin_amdgcn_exp2f(-A.alpha_l2e * (z - zref)) * invS;
    const float l = s * (Tb - A.alpha * (z - zref));
    const float iz = 1.f / z;
    const float v0 = dx * iz, v1 = dy * iz, v2 = dz * iz;
    V0 = fmaf(s, v0, V0);
    V1 = fmaf(s, v1, V1);
    V2 = fmaf(s, v2, V2);
    G0 = fmaf(l, v0, G0);
    G1 = fmaf(l, v1, G1);
    G2 = fmaf(l, v2, G2);
  }
  const float a2 = A.alpha * A.alpha;
  float r0 = 0.f, r1 = 0.f, r2 = 0.f;
  for (int i = 0; i < m; ++i) {
    const float4 P = A.ps[b + i];
    const float dx = lx - P.x, dy = ly - P.y, dz = lz - P.z;
    const float z = __builtin_amdgcn_sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
    if (!(z > 0.f)) continue;
    const float s = __builtin_amdgcn_exp2f(-A.alpha_l2e * (z - zref)) * invS;
    const float l = s * (Tb - A.alpha * (z - zref));
    const float iz = 1.f / z;
    const float v0 = dx * iz, v1 = dy * iz, v2 = dz * iz;
    const float sv = A.sv[b + i];
    const float lz2 = (l * iz) * (l * iz);
    const float x0 = l * (v0 - V0) + s * (v0 - G0);
    const float x1 = l * (v1 - V1) + s * (v1 - G1);
    const float x2 = l * (v2 - V2) + s * (v2 - G2);
    r0 = fmaf(sv, fmaf(a2 * x0, x0, lz2 * (1.f - v0 * v0)), r0);
    r1 = fmaf(sv, fmaf(a2 * x1, x1, lz2 * (1.f - v1 * v1)), r1);
    r2 = fmaf(sv, fmaf(a2 * x2, x2, lz2 * (1.f - v2 * v2)), r2);
  }
  return make_float3(r0, r1, r2);
}

// |L^{-1} k|^2 of the GP variance for the 64 lanes at once on the matrix cores:
// V = L^{-1} K with K's columns the lanes' kernel vectors v (zero beyond m, and for
// lanes that do not use this cell), then each column's squared norm.  The 64 x 64
// product runs as 2 x 2 tiles of v_mfma_f32_32x32x2f32 (the row tile of rows 0-31
// needs only k < 32, L^{-1} being lower triangular): lane l supplies A[l mod 32][l div 32]
// = L^{-1}[row][2t + l div 32] and B[l div 32][l mod 32] = K[2t + l div 32][query], and
// receives D[8 (r div 4) + 4 (l div 32) + r mod 4][l mod 32] in register r.  The B
// operand of a k-step comes from the lane's own column or from the other half-wave's
// (one swap of the half-waves per k-step).
typedef float mfma_acc16 __attribute__((ext_vector_type(16)));
__device__ __forceinline__ float mfma_vv(const float* __restrict__ Li, const float (&v)[64]) {
  const int l = threadIdx.x & 63, hi = l >> 5, col = l & 31;
  float res0 = 0.f, res1 = 0.f;
#pragma unroll 1
  for (int C = 0; C < 2; ++C) {   // query columns 32 C .. 32 C + 31 (one tile pair live)
    mfma_acc16 acc0 = {}, acc1 = {};
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      const float x = hi ? v[2 * t] : v[2 * t + 1];
      const float y = __shfl_xor(x, 32, 64);
      const float bop = C == 0 ? (hi ? y : v[2 * t]) : (hi ? v[2 * t + 1] : y);
      const float* colp = Li + (2 * t + hi) * 64;
      if (t < 16) acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(colp[col], bop, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(colp[32 + col], bop, acc1, 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) s = fmaf(acc0[r], acc0[r], fmaf(acc1[r], acc1[r], s));
    s += __shfl_xor(s, 32, 64);
    if (C == 0) res0 = s;
    else res1 = s;
  }
  return hi ? res1 : res0;
}

// The argmin cell's outputs (gradient, GP variance, softmin variance) and every
// output of the query; all lanes of the wave call it together.  MF (wave-shared cells,
// MB = 64): the GP variance's L^{-1} k on the matrix cores (mfma_vv).
template <int MB, bool LANE, bool MF, bool MAT>
__device__ __forceinline__ void query_finish_t(const FastArgs& A, const Pass1& p1) {
  const bool active = (p1.flags & 2) != 0, outside = (p1.flags & 1) != 0;
  const long qi = p1.qi;
  const float qx = p1.qx, qy = p1.qy, qz = p1.qz;
  const int bc = p1.bc;
  const float best = p1.best, bref = p1.bref;
  const float c2 = A.c2;

  // ---- pass 2: argmin cell outputs, wave-uniform over the distinct argmin cells
  float w0 = 0.f, w1 = 0.f, w2 = 0.f, vv = 0.f, var = 0.f;
  float gv0 = 0.f, gv1 = 0.f, gv2 = 0.f;
  bool todo = bc >= 0;
  while (true) {
    int c;
    if constexpr (LANE) {
      // per lane (sparse queries): every lane its own argmin cell, in one round
      if (!__ballot(todo)) break;
      c = todo ? bc : 0;
    } else {
      unsigned key = todo ? (unsigned)bc : 0xffffffffu;
      key = (unsigned)uniform((int)wave_min_u32(key));
      if (key == 0xffffffffu) break;
      c = (int)key;
    }
    const bool mine = todo && bc == c;
    const int b = LANE ? A.offsets[c] : uniform(A.offsets[c]);
    const int m = (LANE ? A.offsets[c + 1] : uniform(A.offsets[c + 1])) - b;
    const float* Lc = A.L + A.loff[c];
    const float4 ctr = A.centre[c];
    const float lx = qx - ctr.x, ly = qy - ctr.y, lz = qz - ctr.z;
    const float c2d = c2 * bref;
    const float ginv = __builtin_amdgcn_exp2f(-c2d);     // exp(-d^2 / 2 l^2)
    const float zref = __builtin_amdgcn_sqrtf(bref);
    // Far from the cell the exponent c2 (d^2 - z_i^2) is a small difference of large
    // squares, and its FP32 rounding (about eps c2 z^2 per sample) tilts the direction
    // w/|w|.  There it is formed as c2 (d^2 - |l|^2) + c2 (2 l.p_i - |p_i|^2): the
    // first part's rounding is common to every sample and cancels in the direction,
    // the per-sample part is small.  Near the cell the direct form is the accurate one.
    const float ll = fmaf(lz, lz, fmaf(ly, ly, lx * lx));
    const bool farl = ll > A.far2;
    const float k0 = c2 * (bref - ll);
    const float tx = 2.f * c2 * lx, ty = 2.f * c2 * ly, tz = 2.f * c2 * lz;
    // Matern: e_i = e^{-c (z_i - zref)}, far from the cell through zref - z_i =
    // ((bref - |l|^2) + 2 l.p_i - |p_i|^2) / (zref + z_i), and k_i = (1 + c z_i) e_i e^{-c zref}
    constexpr bool mat = MAT;
    const float ginvm = mat ? __builtin_amdgcn_exp2f(-A.mc_l2e * zref) : 0.f;
    const float bm = bref - ll;
    static_assert(!MF || (MB == 64 && !LANE), "the matrix-core GP variance needs m <= 64");
    float v[MB];
    if constexpr (MF) {
#pragma unroll
      for (int i = 0; i < MB; ++i) v[i] = 0.f;
    }
    if (mine) {
      // samples per load group: 8 through scalar registers, 2 when each lane loads
      // its own cell into vector registers
      constexpr int CHP = LANE ? 2 : CH;
      float S = 0.f, T1 = 0.f, X0 = 0.f, X1 = 0.f, X2 = 0.f;
      float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
      for (int i0 = 0; i0 < MB; i0 += CHP) {
        if (i0 < m) {
          float4 P[CHP];
          float SV[CHP];
#pragma unroll
          for (int j = 0; j < CHP; ++j) {
            P[j] = A.ps[b + i0 + j];
            SV[j] = A.sv[b + i0 + j];
          }
#pragma unroll
          for (int j = 0; j < CHP; ++j) {
            const bool in = i0 + j < m;
            const float aw = P[j].w;
            const float dx = lx - P[j].x, dy = ly - P[j].y, dz = lz - P[j].z;
            const float z2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const float pp = fmaf(P[j].z, P[j].z, fmaf(P[j].y, P[j].y, P[j].x * P[j].x));
            const float z = __builtin_amdgcn_sqrtf(z2);
            float e, kv;
            if constexpr (mat) {
              const float lp2 = fmaf(2.f * lx, P[j].x, fmaf(2.f * ly, P[j].y, fmaf(2.f * lz, P[j].z, bm - pp)));
              const float dd = farl ? lp2 / (zref + z) : zref - z;
              e = in ? __builtin_amdgcn_exp2f(A.mc_l2e * dd) : 0.f;
              kv = fmaf(A.mc, z, 1.f) * e * ginvm;
            } else {
              const float arg_far = fmaf(tx, P[j].x, fmaf(ty, P[j].y, fmaf(tz, P[j].z, fmaf(-c2, pp, k0))));
              const float arg = farl ? arg_far : fmaf(z2, -c2, c2d);
              e = in ? __builtin_amdgcn_exp2f(arg) : 0.f;   // see pass 1
              kv = e * ginv;                                 // k_i = exp(-z_i^2 / 2 l^2)
            }
            const float ae = aw * e;
            a0 = fmaf(ae, dx, a0);
            a1 = fmaf(ae, dy, a1);
            a2 = fmaf(ae, dz, a2);
            v[i0 + j] = in ? kv : 0.f;
            // softmin with t_i = alpha (z_i - zref) >= 0
            const float ti = A.alpha * (z - zref);
            const float sm = in ? __builtin_amdgcn_exp2f(-A.alpha_l2e * (z - zref)) : 0.f;
            const float q = sm * sm * SV[j];
            S += sm;
            T1 = fmaf(sm, ti, T1);
            X0 += q;
            X1 = fmaf(q, ti, X1);
            X2 = fmaf(q * ti, ti, X2);
          }
        }
      }
      if constexpr (!MF) vv = forward_subst<MB, LANE ? 16 : 32>(Lc, m, v);
      const float Tb = 1.f + T1 / S;
      var = (Tb * Tb * X0 - 2.f * Tb * X1 + X2) / (S * S);
      w0 = a0;
      w1 = a1;
      w2 = a2;
      if (A.grad_var) {
        const float3 g = grad_var_cell(A, b, m, lx, ly, lz, zref, S, Tb);
        gv0 = g.x;
        gv1 = g.y;
        gv2 = g.z;
      }
      todo = false;
    }
    if constexpr (MF) {
      const float vm = mfma_vv(A.Linv + 4096L * c, v);
      if (mine) vv = vm;
    }
  }

  if (!active) return;
  const float sgn = A.sign ? (float)A.sign[qi] : 1.f;
  uint8_t st = outside ? KSDF_Q_OUTSIDE_INDEX : 0;
  if (p1.flags & PASS1_FIT_TIMEOUT) st |= KSDF_Q_FIT_TIMEOUT;
  if (bc < 0) {
    if (A.grad_var) {
      A.grad_var[3 * qi] = INFINITY;
      A.grad_var[3 * qi + 1] = INFINITY;
      A.grad_var[3 * qi + 2] = INFINITY;
    }
    A.mean[qi] = INFINITY;
    A.grad[3 * qi] = 0.f;
    A.grad[3 * qi + 1] = 0.f;
    A.grad[3 * qi + 2] = 0.f;
    A.var[qi] = INFINITY;
    if (A.var_f) A.var_f[qi] = 1.f;
    if (A.argmin) A.argmin[qi] = -1;
    if (A.qst) A.qst[qi] = st | KSDF_Q_NO_VALID_CELL;
    return;
  }
  float u = 0.f;
  if (best < 0.f) st |= KSDF_Q_CLAMPED;
  else u = MAT ? best : sqrtf(best);   // Matern records carry u, RBF u^2
  const float wn = sqrtf(w0 * w0 + w1 * w1 + w2 * w2);
  float gx = 0.f, gy = 0.f, gz = 0.f;
  if (wn > 0.f) {
    gx = w0 / wn;
    gy = w1 / wn;
    gz = w2 / wn;
  } else {
    st |= KSDF_Q_GRAD_ZERO;
  }
  A.mean[qi] = sgn * u;
  A.grad[3 * qi] = sgn * gx;
  A.grad[3 * qi + 1] = sgn * gy;
  A.grad[3 * qi + 2] = sgn * gz;
  A.var[qi] = var;
  if (A.var_f) A.var_f[qi] = fmaxf(1.f - vv, 0.f);
  if (A.grad_var) {
    A.grad_var[3 * qi] = gv0;
    A.grad_var[3 * qi + 1] = gv1;
    A.grad_var[3 * qi + 2] = gv2;
  }
  if (A.argmin) A.argmin[qi] = bc;
  if (A.qst) A.qst[qi] = st;
}

// The whole query for one wave of sorted queries (MAT: a Matern model).
template <int KM, int MB, bool MAT = false>
__device__ __forceinline__ void query_tile(const FastArgs& A, long sq) {
  query_finish_t<MB, false, false, MAT>(A, query_pass1<KM, false, MAT>(A, sq));
}

// ---------------------------------------------------------------------------
// bucketing: histogram, scan, scatter
// ---------------------------------------------------------------------------
__global__ void fill_kernel(int* p, long n, int v) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// The counting sort's count and scatter take one atomic per distinct key of a wave
// (wave_count, wave_slot): consecutive queries mostly share their bins.
__global__ void bin_kernel(FastArgs A, int* keys, int* counts, long n_bins) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = q < A.Q;
  int key = 0;
  if (valid) {
    int sub;
    const long b = box_key(A, A.pts[3 * q], A.pts[3 * q + 1], A.pts[3 * q + 2], &sub);
    key = b < 0 ? (int)(n_bins - 1) : (int)((long)A.box_rank[b] * A.sub * A.sub * A.sub + sub);
    keys[q] = key;
  }
  wave_count(counts, key, valid);
}

constexpr int SCAN_T = 256;
constexpr int SCAN_PER = 16;
constexpr int SCAN_TILE = SCAN_T * SCAN_PER;

__global__ void __launch_bounds__(SCAN_T) scan_tiles_kernel(const int* in, long n, int* tile_sum) {
  __shared__ int red[SCAN_T];
  const long base = (long)blockIdx.x * SCAN_TILE;
  int s = 0;
  for (int j = 0; j < SCAN_PER; ++j) {
    const long i = base + (long)threadIdx.x * SCAN_PER + j;
    if (i < n) s += in[i];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = SCAN_T / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = red[0];
}

// exclusive scan of the tile sums in one block (n_tiles <= SCAN_T * SCAN_PER)
__global__ void __launch_bounds__(SCAN_T) scan_sums_kernel(int* tile_sum, int n_tiles) {
  __shared__ int part[SCAN_T];
  int v[SCAN_PER];
  int s = 0;
  for (int j = 0; j < SCAN_PER; ++j) {
    const int i = threadIdx.x * SCAN_PER + j;
    v[j] = i < n_tiles ? tile_sum[i] : 0;
    s += v[j];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < SCAN_T; o <<= 1) {
    const int t = (int)threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += t;
    __syncthreads();
  }
  int run = part[threadIdx.x] - s;
  for (int j = 0; j < SCAN_PER; ++j) {
    const int i = threadIdx.x * SCAN_PER + j;
    if (i < n_tiles) tile_sum[i] = run;
    run += v[j];
  }
}

__global__ void __launch_bounds__(SCAN_T) scan_apply_kernel(const int* in, long n,
                                                            const int* tile_off, int* out) {
  __shared__ int part[SCAN_T];
  const long base = (long)blockIdx.x * SCAN_TILE + (long)threadIdx.x * SCAN_PER;
  int v[SCAN_PER];
  int s = 0;
  for (int j = 0; j < SCAN_PER; ++j) {
    v[j] = (base + j < n) ? in[base + j] : 0;
    s += v[j];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < SCAN_T; o <<= 1) {
    const int t = (int)threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += t;
    __syncthreads();
  }
  int run = tile_off[blockIdx.x] + part[threadIdx.x] - s;
  for (int j = 0; j < SCAN_PER; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
}

__global__ void scatter_kernel(long Q, const int* keys, int* cursor, int* perm) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = q < Q;
  const int pos = wave_slot(cursor, valid ? keys[q] : 0, valid);
  if (valid) perm[pos] = (int)q;
}

// bucketing granularity (sub-boxes per box edge): the tuned value, else the finest
// that keeps the bin count near 8M
int sub_of(const ksdf_model* m) {
  const long nb = m->index.n_boxes;
  const int t = m->tuning.query_sub;
  if ((t == 1 || t == 2 || t == 4) && nb * t * t * t <= (16L << 20)) return t;
  return nb * 64 <= (8L << 20) ? 4 : (nb * 8 <= (8L << 20) ? 2 : 1);
}
long n_bins_of(const ksdf_model* m) {
  const long s = sub_of(m);
  return m->index.n_boxes * s * s * s + 1;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }


// Query arguments of an FP32 model (outputs set by the caller's launch).
inline FastArgs make_fast_args(const ksdf_model* m, const void* points, long Q, const int8_t* sign,
                               void* mean, void* grad, void* var, void* var_f, void* grad_var, int* argmin,
                               uint8_t* q_status) {
  FastArgs A{};
  A.pts = static_cast<const float*>(points);
  A.Q = Q;
  A.sign = sign;
  A.mean = static_cast<float*>(mean);
  A.grad = static_cast<float*>(grad);
  A.var = static_cast<float*>(var);
  A.var_f = static_cast<float*>(var_f);
  A.grad_var = static_cast<float*>(grad_var);
  A.argmin = argmin;
  A.qst = q_status;
  A.n_cells = m->n_cells;
  A.k = std::min(m->k_fuse, m->n_cells);
  A.offsets = m->offsets;
  A.loff = m->loff;
  A.ps = reinterpret_cast<const float4*>(m->ps32);
  A.plo = reinterpret_cast<const float4*>(m->plo32);
  A.sv = m->sv32;
  A.L = m->L32;
  A.Linv = m->Linv32;
  A.p2rank = m->max_m > 64 ? m->bucket_rank : nullptr;
  A.centre = reinterpret_cast<const float4*>(m->centre32);
  A.box = m->box32;
  for (int d = 0; d < 3; ++d) {
    A.origin[d] = (float)m->origin[d];
    A.lo[d] = m->index.lo[d];
    A.dims[d] = m->index.dims[d];
  }
  A.inv_h = (float)(1.0 / m->h);
  A.sub = sub_of(m);
  A.n_boxes = m->index.n_boxes;
  A.box_off = m->index.box_off;
  A.box_rank = m->index.box_rank;
  A.box_list = m->index.box_list;
  const double two_l2 = 2.0 * m->ell * m->ell;
  A.c2 = (float)(1.4426950408889634 / two_l2);
  A.two_l2 = (float)two_l2;
  A.alpha = (float)m->alpha;
  A.alpha_l2e = (float)(m->alpha * 1.4426950408889634);
  A.far2 = (float)(4.0 * m->h * m->h);
  const double inv = 1.0 / two_l2;
  A.inv2l2_ff[0] = (float)inv;
  A.inv2l2_ff[1] = (float)(inv - (double)(float)inv);
  A.two_l2_ff[0] = (float)two_l2;
  A.two_l2_ff[1] = (float)(two_l2 - (double)(float)two_l2);
  A.matern = m->kernel == KSDF_KERNEL_MATERN32 ? 1 : 0;
  const double mc = std::sqrt(3.0) / m->ell;
  A.mc = (float)mc;
  A.mc_l2e = (float)(mc * 1.4426950408889634);
  A.mc_ff[0] = (float)mc;
  A.mc_ff[1] = (float)(mc - (double)(float)mc);
  A.inv_mc_ff[0] = (float)(1.0 / mc);
  A.inv_mc_ff[1] = (float)(1.0 / mc - (double)(float)(1.0 / mc));
  return A;
}

// The permutation written by launch_bucketing (the workspace's second array).
inline int* bucketed_perm(void* ws, long Q) {
  return reinterpret_cast<int*>(static_cast<char*>(ws) + align256(Q * sizeof(int)));
}

// Counting sort of the queries by (index box, sub-box); sets A.perm.
inline int launch_bucketing(const ksdf_model* m, FastArgs& A, void* ws, hipStream_t s) {
  const long Q = A.Q;
  // workspace carve-up
  const long nb = n_bins_of(m);
  const long tiles = (nb + SCAN_TILE - 1) / SCAN_TILE;
  char* w = static_cast<char*>(ws);
  int* keys = reinterpret_cast<int*>(w);
  w += align256(Q * sizeof(int));
  int* perm = reinterpret_cast<int*>(w);
  w += align256(Q * sizeof(int));
  int* counts = reinterpret_cast<int*>(w);
  w += align256(nb * sizeof(int));
  int* cursor = reinterpret_cast<int*>(w);
  w += align256(nb * sizeof(int));
  int* tsum = reinterpret_cast<int*>(w);
  if (tiles > (long)SCAN_TILE) {
    set_error("query bucketing: too many bins");
    return KSDF_ERR_UNSUPPORTED;
  }

  const unsigned g1 = (unsigned)((Q + 255) / 256);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, counts, nb, 0);
  hipLaunchKernelGGL(bin_kernel, dim3(g1), dim3(256), 0, s, A, keys, counts, nb);
  hipLaunchKernelGGL(scan_tiles_kernel, dim3((unsigned)tiles), dim3(SCAN_T), 0, s, counts, nb, tsum);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(SCAN_T), 0, s, tsum, (int)tiles);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)tiles), dim3(SCAN_T), 0, s, counts, nb, tsum, cursor);
  hipLaunchKernelGGL(scatter_kernel, dim3(g1), dim3(256), 0, s, Q, keys, cursor, perm);
  A.perm = perm;
  return KSDF_OK;
}

}  // namespace
}  // namespace ksdf
