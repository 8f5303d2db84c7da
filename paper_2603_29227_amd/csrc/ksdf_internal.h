// Internal declarations shared by the ksdf HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ksdf.h"

namespace ksdf {

// Padding (entries) after the FP32 per-sample arrays and after the packed factors,
// so chunked loads past the last cell stay inside the allocation.
#define KSDF_PAD_SAMPLES 16
#define KSDF_PAD_FACTOR 64

// Per-thread error message behind ksdf_last_error().
void set_error(const std::string& msg);

#define KSDF_HIP_TRY(expr)                                                              \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess) {                                                             \
      ::ksdf::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));            \
      return KSDF_ERR_HIP;                                                              \
    }                                                                                   \
  } while (0)

// Candidate index over a lattice of cell-sized boxes: for lattice box B, every
// occupied cell that can be among the K nearest cell centres of some point of B.
struct CandidateIndex {
  int lo[3] = {0, 0, 0};       // lattice key of box (0,0,0)
  int dims[3] = {0, 0, 0};
  long n_boxes = 0;
  long entries = 0;
  int* box_off = nullptr;      // [n_boxes+1]
  int* box_list = nullptr;     // [entries] cell ids, ascending within a box
  int* box_rank = nullptr;     // [n_boxes] position of each box in Z (Morton) order
  int* kmap = nullptr;         // [n_boxes] cell id at each lattice key, -1 where none
  long* bound = nullptr;       // [n_boxes] inclusion bound on near distances, (h/2)^2 units
  int* counts = nullptr;       // [n_boxes] list lengths (count pass)
  int max_list = 0;
};

}  // namespace ksdf

// The model: per-cell store and candidate index, views into caller-owned device
// memory (the store buffer and the index list buffer).
struct ksdf_model {
  int device = 0;
  int n_cu = 0;  // compute units of the device
  int precision = KSDF_FP32;
  int kernel = KSDF_KERNEL_RBF;
  int k_fuse = 8;
  int n_cells = 0;
  long nnz = 0;
  int max_m = 0;
  long n_points = 0;
  double origin[3] = {0, 0, 0};

  double h = 0;
  double ell = 0, noise_var = 0, alpha = 0;   // of the last fit
  double cond_thr = 1e6;
  bool alpha_tied = true;
  bool fitted = false;
  bool has_svar = false;

  std::vector<int> h_offsets;   // host copy of the CSR offsets
  std::vector<long> h_loff;     // host copy of packed-factor offsets
  std::vector<double> h_centre; // host copy of the cell centres [n,3]
  std::vector<int> h_keys;      // host copy of the cell keys [n,3]

  // structure (device)
  int* offsets = nullptr;       // [n+1]
  int* samples = nullptr;       // [nnz] global sample ids
  long* loff = nullptr;         // [n+1] packed lower-triangle offsets, m(m+1)/2 each
  float* centre32 = nullptr;    // [n,4] centre xyz (exact), pad
  double* centre64 = nullptr;   // [n,3]

  // FP32 store (KSDF_FP32 models)
  float* ps32 = nullptr;        // [nnz,4] cell-local (px,py,pz) and weight a
  float* plo32 = nullptr;       // [nnz,4] float-float low parts of ps32
  float* sv32 = nullptr;        // [nnz] sample variance sigma_i^2
  float* L32 = nullptr;         // packed rows of L; diagonal holds 1/L_jj
  float* Linv32 = nullptr;      // [n,64,64] dense L^{-1}, column-major, zero-padded (max m <= 64)
  mutable bool linv_ok = false; // Linv32 holds the inverse of the current L32
  float* box32 = nullptr;       // [n,8] sample AABB lo xyz, A+ (sum of positive a), hi xyz, pad
  float* cond32 = nullptr;      // [n] condition estimate (FP32 factor)
  int* fb_list = nullptr;       // [n] cells to refit in FP64
  int* fb_count = nullptr;      // [1]

  // FP64 store (KSDF_FP64 models, and FP64 refits of FP32 models)
  double* ps64 = nullptr;       // [nnz,4]
  double* sv64 = nullptr;       // [nnz]
  double* L64 = nullptr;        // packed rows of L; diagonal holds 1/L_jj

  uint8_t* cstatus = nullptr;   // [n] KSDF_C_* bits of the last fit
  // adjoint of the fit (prepared when the hyperparameters ask for it)
  bool adjoint_alloc = false;   // storage for the adjoint vectors exists
  bool adjoint_varf_alloc = false;
  bool adjoint = false;         // xi vectors prepared by the last fit
  bool adjoint_varf = false;    // packed dA/dl prepared by the last fit
  float* xi32 = nullptr;        // [nnz+pad,4] xi_l = A^{-1}(dA/dl)a, xi_s = A^{-1}a (float-float)
  double* xi64 = nullptr;       // [nnz,2] (FP64 models)
  float* D32 = nullptr;         // packed dA/dl (FP32 models)
  double* D64 = nullptr;        // packed dA/dl (FP64 models)
  int* bucket_cells = nullptr;  // [n] cell ids grouped by m bucket (<=16, <=32, <=64, <=128)
  int* bucket_rank = nullptr;   // [n] position of each cell in bucket_cells
  int* fused_order = nullptr;   // [n] cell ids by m descending (fused launch fit order)
  int bucket_start[5] = {0, 0, 0, 0, 0};

  ksdf::CandidateIndex index;
  ksdf_tuning tuning{0, 256, 1, 16, 1, 0, 0, 0, 0};
  bool dense_inv = false;       // the store holds Linv32 (KSDF_FIT_DENSE_INV)
  int* flags = nullptr;         // [1] (store) bit 0: a fused launch's wait for the fits expired
  long wait_limit = 1L << 26;   // sleeps before the fused launch's wait gives up
  bool index_ready = false;     // the candidate lists are attached and filled
  size_t store_bytes = 0;
  // kernel timing: one event pair per phase, recorded when timing is on
  bool timing = false;
  hipEvent_t tev[KSDF_TIMER_COUNT][KSDF_TIMER_SLOTS][2] = {};
  mutable int tcount[KSDF_TIMER_COUNT] = {};   // launches since the last read
  size_t device_bytes = 0;
  // second stream (default priority) for the query bucketing beside the fit in
  // ksdf_fit_query, with its fork and join events; null when it could not be made
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

namespace ksdf {
// record the start (end=0) or end (end=1) event of a timed phase
inline void timer_mark(const ksdf_model* m, int which, int end, hipStream_t s) {
  if (!m->timing) return;
  (void)hipEventRecord(m->tev[which][m->tcount[which] % KSDF_TIMER_SLOTS][end], s);
  if (end) ++m->tcount[which];
}
}  // namespace ksdf

namespace ksdf {

// launchers (each returns KSDF_OK or an error after setting the message)
int launch_fit(ksdf_model* m, const void* pts, int dtype, const void* svar, uint8_t* user_status,
               hipStream_t s);
// dense L^{-1} per cell from the FP32 store's factor, for the matrix-core pass 2:
// computed after each fit while query_mfma is on, else marked stale (and then
// computed by the first query that needs it)
void launch_linv(const ksdf_model* m, hipStream_t s);
// candidate index: lattice from the cell centres and the query box (host), the
// count pass (fixes entries; synchronises the stream) and the fill pass (needs
// index.box_list)
int index_lattice(ksdf_model* m, const double* qlo, const double* qhi);
int index_count(ksdf_model* m, hipStream_t s);
int index_fill(ksdf_model* m, hipStream_t s);
// sign from BHM weights
size_t bhm_tau_workspace_bytes(long K);
int launch_bhm_sign(const ksdf_bhm_layout* L, const int* box_bhm, const double* weights,
                    const void* points, int dtype, long Q, double tau, int8_t* sign,
                    double* logodds, hipStream_t s);
int launch_bhm_update_tau(const ksdf_bhm_layout* L, const int* box_bhm, const double* weights,
                          const void* hits, int dtype, long K, double alpha, double* tau, void* ws,
                          size_t ws_bytes, hipStream_t s);
// streaming refit of the highest-priority dirty cells and the query counter update
size_t refit_workspace_bytes(const ksdf_model* m, int budget);
int launch_refit(ksdf_model* m, const void* pts, int dtype, const void* svar, float* dirty,
                 float* qcount, double eta, int budget, int* sel, int* n_sel, uint8_t* user_status,
                 void* ws, hipStream_t s);
size_t count_queries_workspace_bytes(const ksdf_model* m);
int launch_count_queries(const ksdf_model* m, const int* argmin, long Q, float* qcount, float cap,
                         void* ws, hipStream_t s);
// prebucketed: the workspace already holds launch_query_bucketing's sort of these
// points (FP32 models), so the query starts after it
int launch_query(const ksdf_model* m, const void* points, long Q, const int8_t* sign, void* mean,
                 void* grad, void* var, void* var_f, void* grad_var, int* argmin, uint8_t* q_status, void* ws,
                 size_t ws_bytes, hipStream_t s, bool prebucketed = false);
size_t query_workspace_bytes(const ksdf_model* m, long Q);
// The query's bucketing alone (the first step of launch_query_fast), for running it
// beside the fit; launch_query_fast then skips it when called with prebucketed set.
int launch_query_bucketing(const ksdf_model* m, const void* points, long Q, void* ws, hipStream_t s);
int launch_query_fast(const ksdf_model* m, const void* points, long Q, const int8_t* sign,
                      void* mean, void* grad, void* var, void* var_f, void* grad_var, int* argmin,
                      uint8_t* q_status, void* ws, size_t ws_bytes, hipStream_t s,
                      bool prebucketed = false);
size_t query_fast_workspace_bytes(const ksdf_model* m, long Q);
// the softplus margin cost whose mean/var cotangents ksdf_cost_backward forms in the
// backward kernel (device arrays of the model's precision)
struct CostArgs {
  const void* mean;
  const void* var;
  double margin, kvar;
  void* cost;
};
int launch_backward(const ksdf_model* m, const void* points, long Q, const int8_t* sign,
                    const int* argmin, const void* d_mean, const void* d_grad, const void* d_var,
                    const void* d_var_f, void* d_points, double* d_hyper, void* ws,
                    size_t ws_bytes, hipStream_t s,
                    const CostArgs* cost = nullptr);
size_t backward_workspace_bytes(const ksdf_model* m, long Q);
size_t fused_workspace_bytes(const ksdf_model* m, long Q);
int launch_fit_query_fused(ksdf_model* m, const void* pts, int dtype, const void* svar,
                           uint8_t* cell_status, const void* points, long Q, const int8_t* sign,
                           void* mean, void* grad, void* var, void* var_f, void* grad_var, int* argmin,
                           uint8_t* q_status, void* ws, size_t ws_bytes, hipStream_t s);

}  // namespace ksdf
