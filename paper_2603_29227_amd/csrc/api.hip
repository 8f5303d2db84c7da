// C ABI of libksdf: argument checking, model memory, launches.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "ksdf_internal.h"

namespace ksdf {

namespace {
thread_local std::string g_last_error;

bool finite3(const double* v) {
  return v && std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

int check_hyper(const ksdf_hyper* hp) {
  if (!hp) {
    set_error("hyperparameters are null");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  if (!std::isfinite(hp->ell) || !std::isfinite(hp->noise_var) || !std::isfinite(hp->alpha) ||
      !std::isfinite(hp->cond_fp64_threshold)) {
    set_error("non-finite hyperparameter");
    return KSDF_ERR_INVALID_INPUT;
  }
  if (!(hp->ell > 0) || hp->noise_var < 0 || hp->k_fuse < 1 || hp->k_fuse > KSDF_MAX_K ||
      (hp->precision != KSDF_FP64 && hp->precision != KSDF_FP32) ||
      !(hp->cond_fp64_threshold > 0) || (hp->flags & ~(KSDF_FIT_ADJOINT | KSDF_FIT_ADJOINT_VARF | KSDF_FIT_DENSE_INV)) ||
      (hp->kernel != KSDF_KERNEL_RBF && hp->kernel != KSDF_KERNEL_MATERN32)) {
    set_error("hyperparameter out of range (ell > 0, noise_var >= 0, 1 <= k_fuse <= 16, "
              "precision KSDF_FP64|KSDF_FP32, cond threshold > 0, kernel KSDF_KERNEL_*)");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  return KSDF_OK;
}

int check_device(const ksdf_model* m) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != m->device) {
    set_error("the current device is not the model's device");
    return KSDF_ERR_DEVICE;
  }
  return KSDF_OK;
}

// Lays the model's device arrays out in one caller buffer, 256-byte aligned; with a
// null base it only adds up the bytes.  model_layout below is the single place that
// decides the layout, used both to size the store and to carve it.
struct Carver {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  void take(T** p, size_t n) {
    off = (off + 255) & ~size_t(255);
    *p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += std::max<size_t>(n, 1) * sizeof(T);
  }
};

void model_layout(ksdf_model* m, Carver& cv) {
  const long n = m->n_cells, nnz = m->nnz, lsize = m->h_loff[m->n_cells];
  cv.take(&m->offsets, n + 1);
  cv.take(&m->samples, nnz);
  cv.take(&m->loff, n + 1);
  cv.take(&m->centre32, 4 * n);
  cv.take(&m->centre64, 3 * n);
  cv.take(&m->box32, 8 * n);
  cv.take(&m->cstatus, n);
  cv.take(&m->ps64, 4 * nnz);
  cv.take(&m->sv64, nnz);
  cv.take(&m->L64, lsize);
  cv.take(&m->bucket_cells, n);
  cv.take(&m->bucket_rank, n);
  cv.take(&m->fused_order, n);
  cv.take(&m->flags, 1);
  if (m->adjoint_alloc) {
    // the FP64 refit of an FP32 model writes its xi in FP32 too
    if (m->precision == KSDF_FP32) cv.take(&m->xi32, 4 * (nnz + KSDF_PAD_SAMPLES));
    else cv.take(&m->xi64, 2 * nnz);
  }
  if (m->adjoint_varf_alloc) {
    if (m->precision == KSDF_FP32) cv.take(&m->D32, lsize + KSDF_PAD_FACTOR);
    else cv.take(&m->D64, lsize);
  }
  if (m->precision == KSDF_FP32) {
    // padded so the wave-uniform chunked loads of the last cell stay in bounds
    cv.take(&m->ps32, 4 * (nnz + KSDF_PAD_SAMPLES));
    cv.take(&m->plo32, 4 * (nnz + KSDF_PAD_SAMPLES));
    cv.take(&m->sv32, nnz + KSDF_PAD_SAMPLES);
    cv.take(&m->L32, lsize + KSDF_PAD_FACTOR);
    cv.take(&m->cond32, n);
    cv.take(&m->fb_list, n);
    cv.take(&m->fb_count, 1);
    if (m->dense_inv) cv.take(&m->Linv32, 4096 * n);
  }
  const long nb = m->index.n_boxes;
  cv.take(&m->index.box_off, nb + 1);
  cv.take(&m->index.box_rank, nb);
  cv.take(&m->index.kmap, nb);
  cv.take(&m->index.bound, nb);
  cv.take(&m->index.counts, nb);
}

// Host part of model creation, shared by ksdf_model_bytes and ksdf_model_create:
// argument checks, sizes, host copies of the structure and the index lattice.
int model_host_setup(ksdf_model* m, int n_cells, const int* offsets, const int* samples,
                     const int* keys, const double origin[3], double h, long n_points,
                     const ksdf_hyper* hyper, const double query_lo[3], const double query_hi[3]) {
  int r = check_hyper(hyper);
  if (r) return r;
  if (n_cells >= (1 << 28) - 1) {
    set_error("ksdf_model_create: more than 2^28 - 2 cells");
    return KSDF_ERR_UNSUPPORTED;
  }
  if (n_cells < 0 || !offsets || (n_cells > 0 && (!samples || !keys)) || !finite3(origin) ||
      !(h > 0) || n_points < 0 || ((query_lo == nullptr) != (query_hi == nullptr))) {
    set_error("ksdf_model_create: invalid argument");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  if (query_lo && (!finite3(query_lo) || !finite3(query_hi))) {
    set_error("ksdf_model_create: non-finite query box");
    return KSDF_ERR_INVALID_INPUT;
  }
  if (offsets[0] != 0) {
    set_error("offsets[0] must be 0");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  int max_m = 0;
  for (int c = 0; c < n_cells; ++c) {
    const int mc = offsets[c + 1] - offsets[c];
    if (mc < 1) {
      set_error("every cell needs at least one sample");
      return KSDF_ERR_INVALID_ARGUMENT;
    }
    if (mc > KSDF_MAX_M) {
      set_error("a cell has more than 128 samples");
      return KSDF_ERR_UNSUPPORTED;
    }
    max_m = std::max(max_m, mc);
  }
  // the candidate index visits keys in order and must meet cell ids ascending
  for (int c = 1; c < n_cells; ++c) {
    const int* a = keys + 3L * (c - 1);
    const int* b = keys + 3L * c;
    if (!std::lexicographical_compare(a, a + 3, b, b + 3)) {
      set_error("cell keys must be unique and in lexicographic order (as the cell builder writes them)");
      return KSDF_ERR_INVALID_ARGUMENT;
    }
  }
  const long nnz = offsets[n_cells];
  for (long i = 0; i < nnz; ++i)
    if (samples[i] < 0 || samples[i] >= n_points) {
      set_error("a cell references a sample index outside [0, n_points)");
      return KSDF_ERR_INVALID_ARGUMENT;
    }
  m->precision = hyper->precision;
  m->kernel = hyper->kernel;
  m->k_fuse = hyper->k_fuse;
  m->cond_thr = hyper->cond_fp64_threshold;
  m->n_cells = n_cells;
  m->nnz = nnz;
  m->max_m = max_m;
  m->n_points = n_points;
  for (int d = 0; d < 3; ++d) m->origin[d] = origin[d];
  m->h = h;
  m->h_offsets.assign(offsets, offsets + n_cells + 1);
  m->h_loff.assign(n_cells + 1, 0);
  for (int c = 0; c < n_cells; ++c) {
    const long mc = offsets[c + 1] - offsets[c];
    m->h_loff[c + 1] = m->h_loff[c] + mc * (mc + 1) / 2;
  }
  m->h_keys.assign(keys, keys + 3L * n_cells);
  m->h_centre.resize(3L * n_cells);
  for (int c = 0; c < n_cells; ++c)
    for (int d = 0; d < 3; ++d) m->h_centre[3 * c + d] = origin[d] + ((double)keys[3 * c + d] + 0.5) * h;
  m->adjoint_alloc = (hyper->flags & (KSDF_FIT_ADJOINT | KSDF_FIT_ADJOINT_VARF)) != 0;
  m->adjoint_varf_alloc = (hyper->flags & KSDF_FIT_ADJOINT_VARF) != 0;
  // the dense inverses serve the matrix-core pass 2 of FP32 RBF models with m <= 64
  m->dense_inv = (hyper->flags & KSDF_FIT_DENSE_INV) && m->precision == KSDF_FP32 &&
                 m->kernel == KSDF_KERNEL_RBF && max_m <= 64 && n_cells > 0;
  return index_lattice(m, query_lo, query_hi);
}

void destroy_model(ksdf_model* m) {
  if (!m) return;
  for (auto& phase : m->tev)
    for (auto& pair : phase)
      for (hipEvent_t e : pair)
        if (e) (void)hipEventDestroy(e);
  if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
  if (m->ev_join) (void)hipEventDestroy(m->ev_join);
  if (m->aux) (void)hipStreamDestroy(m->aux);
  delete m;
}

// The model's second stream and its fork/join events; on any failure the model runs
// every step on the caller's stream.
void make_aux_stream(ksdf_model* m) {
  if (hipStreamCreateWithFlags(&m->aux, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&m->ev_join, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
    if (m->ev_join) (void)hipEventDestroy(m->ev_join);
    if (m->aux) (void)hipStreamDestroy(m->aux);
    m->aux = nullptr;
    m->ev_fork = m->ev_join = nullptr;
  }
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace ksdf

using namespace ksdf;

extern "C" size_t ksdf_model_bytes(int n_cells, const int* offsets, const int* samples,
                                   const int* keys, const double origin[3], double h,
                                   long n_points, const ksdf_hyper* hyper,
                                   const double query_lo[3], const double query_hi[3]) {
  ksdf_model m;
  if (model_host_setup(&m, n_cells, offsets, samples, keys, origin, h, n_points, hyper, query_lo,
                       query_hi) != KSDF_OK)
    return 0;
  Carver cv;
  model_layout(&m, cv);
  return cv.off;
}

extern "C" int ksdf_model_create(int n_cells, const int* offsets, const int* samples,
                                 const int* keys, const double origin[3], double h,
                                 long n_points, const ksdf_hyper* hyper, const double query_lo[3],
                                 const double query_hi[3], void* store, size_t store_bytes,
                                 void* stream, ksdf_model** out) {
  if (!out) {
    set_error("out is null");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  *out = nullptr;
  auto* m = new ksdf_model;
  int r = model_host_setup(m, n_cells, offsets, samples, keys, origin, h, n_points, hyper, query_lo,
                           query_hi);
  if (r) {
    destroy_model(m);
    return r;
  }
  Carver size;
  model_layout(m, size);
  if (!store || store_bytes < size.off) {
    destroy_model(m);
    set_error("ksdf_model_create: the store is smaller than ksdf_model_bytes");
    return KSDF_ERR_WORKSPACE;
  }
  if (reinterpret_cast<uintptr_t>(store) % 256 != 0) {
    destroy_model(m);
    set_error("ksdf_model_create: the store must be 256-byte aligned");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    destroy_model(m);
    set_error("no HIP device");
    return KSDF_ERR_DEVICE;
  }
  (void)hipGetDevice(&m->device);
  (void)hipDeviceGetAttribute(&m->n_cu, hipDeviceAttributeMultiprocessorCount, m->device);
  make_aux_stream(m);
  Carver cv;
  cv.base = static_cast<char*>(store);
  model_layout(m, cv);
  m->store_bytes = size.off;
  m->device_bytes = size.off;
  hipStream_t s = (hipStream_t)stream;
  r = [&]() -> int {
    const long nnz = m->nnz, lsize = m->h_loff[n_cells];
    std::vector<float> c32(4L * n_cells, 0.f);
    for (int c = 0; c < n_cells; ++c)
      for (int d = 0; d < 3; ++d) c32[4 * c + d] = (float)m->h_centre[3 * c + d];
    // cells grouped by m bucket for the FP32 fit kernels
    const int edges[4] = {16, 32, 64, 128};
    std::vector<int> order;
    order.reserve(n_cells);
    m->bucket_start[0] = 0;
    for (int bk = 0; bk < 4; ++bk) {
      for (int c = 0; c < n_cells; ++c) {
        const int mc = offsets[c + 1] - offsets[c];
        const int lo = bk == 0 ? 0 : edges[bk - 1];
        if (mc > lo && mc <= edges[bk]) order.push_back(c);
      }
      m->bucket_start[bk + 1] = (int)order.size();
    }
    // fused-launch fit order: largest m first (longest tasks start earliest)
    std::vector<int> byM(order.rbegin(), order.rend());
    std::stable_sort(byM.begin(), byM.end(), [&](int x, int y) {
      return offsets[x + 1] - offsets[x] > offsets[y + 1] - offsets[y];
    });
    auto up = [&](void* dst, const void* src, size_t bytes) -> int {
      if (bytes == 0) return KSDF_OK;
      KSDF_HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
      return KSDF_OK;
    };
    int e;
    if ((e = up(m->offsets, offsets, (n_cells + 1) * sizeof(int)))) return e;
    if ((e = up(m->samples, samples, nnz * sizeof(int)))) return e;
    if ((e = up(m->loff, m->h_loff.data(), (n_cells + 1) * sizeof(long)))) return e;
    if ((e = up(m->centre32, c32.data(), c32.size() * sizeof(float)))) return e;
    if ((e = up(m->centre64, m->h_centre.data(), m->h_centre.size() * sizeof(double)))) return e;
    if ((e = up(m->bucket_cells, order.data(), order.size() * sizeof(int)))) return e;
    std::vector<int> rank(order.size());
    for (size_t i = 0; i < order.size(); ++i) rank[order[i]] = (int)i;
    if ((e = up(m->bucket_rank, rank.data(), rank.size() * sizeof(int)))) return e;
    if ((e = up(m->fused_order, byM.data(), byM.size() * sizeof(int)))) return e;
    KSDF_HIP_TRY(hipMemsetAsync(m->flags, 0, sizeof(int), s));
    if (m->precision == KSDF_FP32) {
      // the padding past the last cell is read by chunked loads: keep it zero
      KSDF_HIP_TRY(hipMemsetAsync(m->ps32, 0, 4L * (nnz + KSDF_PAD_SAMPLES) * sizeof(float), s));
      KSDF_HIP_TRY(hipMemsetAsync(m->sv32, 0, (nnz + KSDF_PAD_SAMPLES) * sizeof(float), s));
      KSDF_HIP_TRY(hipMemsetAsync(m->L32, 0, (lsize + KSDF_PAD_FACTOR) * sizeof(float), s));
    }
    // the index's count pass synchronises the stream, after which the host vectors
    // above may go
    return index_count(m, s);
  }();
  if (r) {
    destroy_model(m);
    return r;
  }
  *out = m;
  return KSDF_OK;
}

extern "C" size_t ksdf_model_index_bytes(const ksdf_model* m) {
  return m ? std::max<long>(m->index.entries, 1) * sizeof(int) : 0;
}

extern "C" int ksdf_model_attach_index(ksdf_model* m, void* list, size_t bytes, void* stream) {
  if (!m || !list || bytes < ksdf_model_index_bytes(m)) {
    set_error("ksdf_model_attach_index: list buffer missing or smaller than ksdf_model_index_bytes");
    return KSDF_ERR_WORKSPACE;
  }
  if (reinterpret_cast<uintptr_t>(list) % 4 != 0) {
    set_error("ksdf_model_attach_index: the list buffer must be 4-byte aligned");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  int r = check_device(m);
  if (r) return r;
  m->index.box_list = static_cast<int*>(list);
  r = index_fill(m, (hipStream_t)stream);
  if (r) return r;
  m->device_bytes = m->store_bytes + ksdf_model_index_bytes(m);
  m->index_ready = true;
  return KSDF_OK;
}

extern "C" int ksdf_model_check(ksdf_model* m, void* stream) {
  if (!m) {
    set_error("ksdf_model_check: model is null");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  int r = check_device(m);
  if (r) return r;
  hipStream_t s = (hipStream_t)stream;
  int flags = 0;
  KSDF_HIP_TRY(hipMemcpyAsync(&flags, m->flags, sizeof(int), hipMemcpyDeviceToHost, s));
  KSDF_HIP_TRY(hipStreamSynchronize(s));
  if (flags & 1) {
    KSDF_HIP_TRY(hipMemsetAsync(m->flags, 0, sizeof(int), s));
    set_error("a fused fit+query launch stopped waiting for the fits; its queries marked "
              "KSDF_Q_FIT_TIMEOUT may have read unfinished cells");
    return KSDF_ERR_TIMEOUT;
  }
  return KSDF_OK;
}

extern "C" int ksdf_model_set_wait_limit(ksdf_model* m, long sleeps) {
  if (!m || sleeps < 0) {
    set_error("ksdf_model_set_wait_limit: invalid argument");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  m->wait_limit = sleeps == 0 ? (1L << 26) : sleeps;
  return KSDF_OK;
}

extern "C" void ksdf_model_destroy(ksdf_model* model) {
  destroy_model(model);
}

extern "C" int ksdf_model_info(const ksdf_model* m, int* n_cells, long* nnz, int* max_m,
                               long* index_entries, size_t* device_bytes) {
  if (!m) return KSDF_ERR_INVALID_ARGUMENT;
  if (n_cells) *n_cells = m->n_cells;
  if (nnz) *nnz = m->nnz;
  if (max_m) *max_m = m->max_m;
  if (index_entries) *index_entries = m->index.entries;
  if (device_bytes) *device_bytes = m->device_bytes;
  return KSDF_OK;
}

namespace {
int prepare_fit(ksdf_model* m, const void* surface_pts, int dtype, long n_points,
                const void* sample_var, const ksdf_hyper* hyper) {
  if (!m) {
    set_error("model is null");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  int r = check_hyper(hyper);
  if (r) return r;
  if ((m->n_cells > 0 && !surface_pts) || (dtype != KSDF_DTYPE_F32 && dtype != KSDF_DTYPE_F64) ||
      n_points != m->n_points || hyper->k_fuse != m->k_fuse || hyper->precision != m->precision ||
      hyper->kernel != m->kernel) {
    set_error("ksdf_fit_cells: arguments do not match the model (n_points, dtype, k_fuse, precision, "
              "kernel)");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  if ((r = check_device(m))) return r;
  const bool want_adj = (hyper->flags & (KSDF_FIT_ADJOINT | KSDF_FIT_ADJOINT_VARF)) != 0;
  const bool want_varf = (hyper->flags & KSDF_FIT_ADJOINT_VARF) != 0;
  if ((want_adj && !m->adjoint_alloc) || (want_varf && !m->adjoint_varf_alloc)) {
    set_error("ksdf_fit_cells: adjoint flags were not requested at ksdf_model_create");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  m->ell = hyper->ell;
  m->noise_var = hyper->noise_var;
  m->alpha_tied = !(hyper->alpha > 0);
  m->alpha = m->alpha_tied ? 1.0 / (2.0 * hyper->ell * hyper->ell) : hyper->alpha;
  m->cond_thr = hyper->cond_fp64_threshold;
  m->has_svar = sample_var != nullptr;
  m->adjoint = want_adj;
  m->adjoint_varf = want_varf;
  return KSDF_OK;
}

int check_query_args(const ksdf_model* m, const void* points, long Q, void* mean, void* grad,
                     void* var) {
  if (!m || Q < 0 || (Q > 0 && (!points || !mean || !grad || !var))) {
    set_error("ksdf_query: invalid argument");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  return KSDF_OK;
}
}  // namespace

extern "C" int ksdf_fit_cells(ksdf_model* m, const void* surface_pts, int dtype, long n_points,
                              const void* sample_var, const ksdf_hyper* hyper,
                              uint8_t* cell_status, void* stream) {
  int r = prepare_fit(m, surface_pts, dtype, n_points, sample_var, hyper);
  if (r) return r;
  r = launch_fit(m, surface_pts, dtype, sample_var, cell_status, (hipStream_t)stream);
  if (r == KSDF_OK) m->fitted = true;
  return r;
}

extern "C" int ksdf_bhm_sign(const ksdf_bhm_layout* layout, const int* box_bhm,
                             const double* weights, const void* points, int dtype, long Q,
                             double tau, int8_t* sign, double* logodds, void* stream) {
  return launch_bhm_sign(layout, box_bhm, weights, points, dtype, Q, tau, sign, logodds,
                         (hipStream_t)stream);
}

extern "C" size_t ksdf_bhm_tau_workspace_bytes(long K) { return K > 0 ? bhm_tau_workspace_bytes(K) : 0; }

extern "C" int ksdf_bhm_update_tau(const ksdf_bhm_layout* layout, const int* box_bhm,
                                   const double* weights, const void* hits, int dtype, long K,
                                   double alpha, double* tau, void* workspace, size_t ws_bytes,
                                   void* stream) {
  return launch_bhm_update_tau(layout, box_bhm, weights, hits, dtype, K, alpha, tau, workspace,
                               ws_bytes, (hipStream_t)stream);
}

extern "C" size_t ksdf_refit_workspace_bytes(const ksdf_model* m, int budget) {
  return (m && budget > 0) ? refit_workspace_bytes(m, budget) : 0;
}

extern "C" int ksdf_refit_cells(ksdf_model* m, const void* surface_pts, int dtype, long n_points,
                                const void* sample_var, float* dirty, float* qcount, double eta,
                                int budget, int* refit_cells, int* n_refit, uint8_t* cell_status,
                                void* workspace, size_t ws_bytes, void* stream) {
  if (!m || !dirty || !qcount || !refit_cells || !n_refit || budget < 1 || !std::isfinite(eta) ||
      eta < 0 || (m->n_cells > 0 && !surface_pts) ||
      (dtype != KSDF_DTYPE_F32 && dtype != KSDF_DTYPE_F64) || n_points != m->n_points) {
    set_error("ksdf_refit_cells: invalid argument");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  if (!m->fitted) {
    set_error("ksdf_refit_cells: the model has not been fitted");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  if (ws_bytes < refit_workspace_bytes(m, budget) || !workspace) {
    set_error("ksdf_refit_cells: workspace too small");
    return KSDF_ERR_WORKSPACE;
  }
  int r = check_device(m);
  if (r) return r;
  return launch_refit(m, surface_pts, dtype, sample_var, dirty, qcount, eta, budget, refit_cells,
                      n_refit, cell_status, workspace, (hipStream_t)stream);
}

extern "C" size_t ksdf_count_queries_workspace_bytes(const ksdf_model* m) {
  return m ? count_queries_workspace_bytes(m) : 0;
}

extern "C" int ksdf_count_queries(const ksdf_model* m, const int* argmin, long Q, float* qcount,
                                  float cap, void* workspace, size_t ws_bytes, void* stream) {
  if (!m || Q < 0 || (Q > 0 && !argmin) || !qcount || !(cap >= 0)) {
    set_error("ksdf_count_queries: invalid argument");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  if (!workspace || ws_bytes < count_queries_workspace_bytes(m)) {
    set_error("ksdf_count_queries: workspace too small");
    return KSDF_ERR_WORKSPACE;
  }
  int r = check_device(m);
  if (r) return r;
  return launch_count_queries(m, argmin, Q, qcount, cap, workspace, (hipStream_t)stream);
}

extern "C" size_t ksdf_fit_query_workspace_bytes(const ksdf_model* m, long Q) {
  if (!m) return 0;
  return m->precision == KSDF_FP32 ? fused_workspace_bytes(m, Q) : query_workspace_bytes(m, Q);
}

extern "C" int ksdf_fit_query(ksdf_model* m, const void* surface_pts, int dtype, long n_points,
                              const void* sample_var, const ksdf_hyper* hyper,
                              uint8_t* cell_status, const void* points, long Q,
                              const int8_t* sign, void* mean, void* grad, void* var, void* var_f, void* grad_var,
                              int* argmin, uint8_t* q_status, void* workspace, size_t ws_bytes,
                              void* stream) {
  int r = prepare_fit(m, surface_pts, dtype, n_points, sample_var, hyper);
  if (r) return r;
  if ((r = check_query_args(m, points, Q, mean, grad, var))) return r;
  if (!m->index_ready) {
    set_error("ksdf_fit_query: the model's index is not attached");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  const size_t need = ksdf_fit_query_workspace_bytes(m, Q);
  if (ws_bytes < need || (need > 0 && !workspace)) {
    set_error("ksdf_fit_query: workspace too small");
    return KSDF_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  if (m->precision == KSDF_FP64) {
    r = launch_fit(m, surface_pts, dtype, sample_var, cell_status, s);
    if (r) return r;
    m->fitted = true;
    return launch_query(m, points, Q, sign, mean, grad, var, var_f, grad_var, argmin, q_status, workspace,
                        ws_bytes, s);
  }
  if (!m->tuning.fused || m->kernel != KSDF_KERNEL_RBF) {
    if (!m->aux || Q == 0) {
      r = launch_fit(m, surface_pts, dtype, sample_var, cell_status, s);
      if (r) return r;
      m->fitted = true;
      return launch_query(m, points, Q, sign, mean, grad, var, var_f, grad_var, argmin, q_status,
                          workspace, ws_bytes, s);
    }
    // The query's bucketing reads only the queries and the candidate index: it runs on
    // the model's second stream beside the fit (which is latency-bound and leaves room
    // on the chip), forked after the caller's earlier work and joined before the query
    // kernels.  Both events are recorded on every path, so a graph capture of the call
    // always joins the second stream back.
    KSDF_HIP_TRY(hipEventRecord(m->ev_fork, s));
    KSDF_HIP_TRY(hipStreamWaitEvent(m->aux, m->ev_fork, 0));
    const int rb = launch_query_bucketing(m, points, Q, workspace, m->aux);
    KSDF_HIP_TRY(hipEventRecord(m->ev_join, m->aux));
    r = launch_fit(m, surface_pts, dtype, sample_var, cell_status, s);
    KSDF_HIP_TRY(hipStreamWaitEvent(s, m->ev_join, 0));
    if (rb) return rb;
    if (r) return r;
    m->fitted = true;
    return launch_query(m, points, Q, sign, mean, grad, var, var_f, grad_var, argmin, q_status, workspace,
                        ws_bytes, s, true);
  }
  r = launch_fit_query_fused(m, surface_pts, dtype, sample_var, cell_status, points, Q, sign,
                             mean, grad, var, var_f, grad_var, argmin, q_status, workspace, ws_bytes, s);
  if (r == KSDF_OK) m->fitted = true;
  return r;
}

extern "C" int ksdf_model_set_tuning(ksdf_model* m, const ksdf_tuning* t) {
  if (!m || !t || (t->query_sub != 0 && t->query_sub != 1 && t->query_sub != 2 && t->query_sub != 4) ||
      (t->query_block != 0 && t->query_block != 64 && t->query_block != 256) ||
      (t->fused != 0 && t->fused != 1) ||
      (t->fit_min_bucket != 16 && t->fit_min_bucket != 32 && t->fit_min_bucket != 64) ||
      (t->query_split != 0 && t->query_split != 1) || (t->query_lanes != 0 && t->query_lanes != 1) ||
      (t->backward_lanes != 0 && t->backward_lanes != 1) || (t->query_pairs != 0 && t->query_pairs != 1) ||
      (t->query_mfma != 0 && t->query_mfma != 1)) {
    set_error("ksdf_model_set_tuning: invalid tuning");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  // the matrix-core pass 2 (two-kernel RBF query of an FP32 model with m <= 64) reads
  // the dense inverses, which the store holds only when created with KSDF_FIT_DENSE_INV
  if (t->query_mfma && !m->dense_inv && m->precision == KSDF_FP32 && m->kernel == KSDF_KERNEL_RBF &&
      m->max_m <= 64 && m->n_cells > 0) {
    set_error("ksdf_model_set_tuning: query_mfma needs a model created with KSDF_FIT_DENSE_INV");
    return KSDF_ERR_UNSUPPORTED;
  }
  m->tuning = *t;
  if (m->tuning.query_block == 0) m->tuning.query_block = 256;
  return KSDF_OK;
}

extern "C" int ksdf_model_set_timing(ksdf_model* m, int on) {
  if (!m) return KSDF_ERR_INVALID_ARGUMENT;
  int r = check_device(m);
  if (r) return r;
  if (on && !m->tev[0][0][0]) {
    for (auto& phase : m->tev)
      for (auto& pair : phase)
        for (hipEvent_t& e : pair) KSDF_HIP_TRY(hipEventCreate(&e));
  }
  m->timing = on != 0;
  for (int& c : m->tcount) c = 0;
  return KSDF_OK;
}

extern "C" int ksdf_model_timer_read(ksdf_model* m, int which, float* ms, int max_n, int* n) {
  if (!m || !n || (max_n > 0 && !ms) || which < 0 || which >= KSDF_TIMER_COUNT || !m->timing) {
    set_error("ksdf_model_timer_read: timing off or bad arguments");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  const int cnt = m->tcount[which];
  m->tcount[which] = 0;
  if (cnt > KSDF_TIMER_SLOTS) {
    set_error("ksdf_model_timer_read: more launches than timer slots since the last read");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  *n = cnt < max_n ? cnt : max_n;
  for (int i = 0; i < *n; ++i) {
    KSDF_HIP_TRY(hipEventSynchronize(m->tev[which][i][1]));
    KSDF_HIP_TRY(hipEventElapsedTime(ms + i, m->tev[which][i][0], m->tev[which][i][1]));
  }
  return KSDF_OK;
}

extern "C" int ksdf_model_get_tuning(const ksdf_model* m, ksdf_tuning* t) {
  if (!m || !t) return KSDF_ERR_INVALID_ARGUMENT;
  *t = m->tuning;
  return KSDF_OK;
}

extern "C" size_t ksdf_query_workspace_bytes(const ksdf_model* m, long Q) {
  return m ? query_workspace_bytes(m, Q) : 0;
}

namespace {
// ksdf_query and ksdf_query_bucketed: argument checks, then the launches
int query_entry(const ksdf_model* m, const void* points, long Q, const int8_t* sign, void* mean,
                void* grad, void* var, void* var_f, void* grad_var, int* argmin, uint8_t* q_status,
                void* workspace, size_t ws_bytes, void* stream, bool prebucketed) {
  if (int r0 = check_query_args(m, points, Q, mean, grad, var)) return r0;
  if (!m->fitted || !m->index_ready) {
    set_error("ksdf_query: the model has not been fitted or its index is not attached");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  const size_t need = query_workspace_bytes(m, Q);
  if (ws_bytes < need || (need > 0 && !workspace)) {
    set_error("ksdf_query: workspace too small");
    return KSDF_ERR_WORKSPACE;
  }
  int r = check_device(m);
  if (r) return r;
  return launch_query(m, points, Q, sign, mean, grad, var, var_f, grad_var, argmin, q_status, workspace,
                      ws_bytes, (hipStream_t)stream, prebucketed && m->precision == KSDF_FP32);
}
}  // namespace

extern "C" int ksdf_query(const ksdf_model* m, const void* points, long Q, const int8_t* sign,
                          void* mean, void* grad, void* var, void* var_f, void* grad_var, int* argmin,
                          uint8_t* q_status, void* workspace, size_t ws_bytes, void* stream) {
  return query_entry(m, points, Q, sign, mean, grad, var, var_f, grad_var, argmin, q_status, workspace,
                     ws_bytes, stream, false);
}

extern "C" int ksdf_query_bucket(const ksdf_model* m, const void* points, long Q, void* workspace,
                                 size_t ws_bytes, void* stream) {
  if (!m || Q < 0 || (Q > 0 && !points)) {
    set_error("ksdf_query_bucket: invalid argument");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  if (!m->index_ready) {
    set_error("ksdf_query_bucket: the model's index is not attached");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  const size_t need = query_workspace_bytes(m, Q);
  if (ws_bytes < need || (need > 0 && !workspace)) {
    set_error("ksdf_query_bucket: workspace too small");
    return KSDF_ERR_WORKSPACE;
  }
  int r = check_device(m);
  if (r) return r;
  if (m->precision != KSDF_FP32 || Q == 0) return KSDF_OK;
  r = launch_query_bucketing(m, points, Q, workspace, (hipStream_t)stream);
  if (r) return r;
  KSDF_HIP_TRY(hipGetLastError());
  return KSDF_OK;
}

extern "C" int ksdf_query_bucketed(const ksdf_model* m, const void* points, long Q,
                                   const int8_t* sign, void* mean, void* grad, void* var,
                                   void* var_f, void* grad_var, int* argmin, uint8_t* q_status,
                                   void* workspace, size_t ws_bytes, void* stream) {
  return query_entry(m, points, Q, sign, mean, grad, var, var_f, grad_var, argmin, q_status, workspace,
                     ws_bytes, stream, true);
}

extern "C" size_t ksdf_backward_workspace_bytes(const ksdf_model* m, long Q) {
  return m ? backward_workspace_bytes(m, Q) : 0;
}

extern "C" int ksdf_query_backward(const ksdf_model* m, const void* points, long Q,
                                   const int8_t* sign, const int* argmin, const void* d_mean,
                                   const void* d_grad, const void* d_var, const void* d_var_f,
                                   void* d_points, double* d_hyper, void* workspace,
                                   size_t ws_bytes, void* stream) {
  if (!m || Q < 0 || (Q > 0 && (!points || !d_points)) || !d_hyper) {
    set_error("ksdf_query_backward: invalid argument");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  if (!m->fitted || !m->index_ready) {
    set_error("ksdf_query_backward: the model has not been fitted or its index is not attached");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  const size_t need = backward_workspace_bytes(m, Q);
  if (ws_bytes < need || (need > 0 && !workspace)) {
    set_error("ksdf_query_backward: workspace too small");
    return KSDF_ERR_WORKSPACE;
  }
  int r = check_device(m);
  if (r) return r;
  return launch_backward(m, points, Q, sign, argmin, d_mean, d_grad, d_var, d_var_f, d_points,
                         d_hyper, workspace, ws_bytes, (hipStream_t)stream);
}

extern "C" int ksdf_cost_backward(const ksdf_model* m, const void* points, long Q,
                                  const int8_t* sign, const int* argmin, const void* mean,
                                  const void* var, double margin, double kvar, void* cost,
                                  void* d_points, double* d_hyper, void* workspace,
                                  size_t ws_bytes, void* stream) {
  if (!m || Q < 0 || (Q > 0 && (!points || !d_points || !mean || !var)) || !d_hyper ||
      !std::isfinite(margin) || !std::isfinite(kvar)) {
    set_error("ksdf_cost_backward: invalid argument");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  if (!m->fitted || !m->index_ready) {
    set_error("ksdf_cost_backward: the model has not been fitted or its index is not attached");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  const size_t need = backward_workspace_bytes(m, Q);
  if (ws_bytes < need || (need > 0 && !workspace)) {
    set_error("ksdf_cost_backward: workspace too small");
    return KSDF_ERR_WORKSPACE;
  }
  int r = check_device(m);
  if (r) return r;
  const CostArgs c{mean, var, margin, kvar, cost};
  return launch_backward(m, points, Q, sign, argmin, nullptr, nullptr, nullptr, nullptr, d_points,
                         d_hyper, workspace, ws_bytes, (hipStream_t)stream, &c);
}

extern "C" const char* ksdf_status_string(int status) {
  switch (status) {
    case KSDF_OK: return "ok";
    case KSDF_ERR_INVALID_ARGUMENT: return "invalid argument";
    case KSDF_ERR_INVALID_INPUT: return "invalid (non-finite) input";
    case KSDF_ERR_WORKSPACE: return "workspace too small";
    case KSDF_ERR_HIP: return "HIP runtime error";
    case KSDF_ERR_DEVICE: return "no usable device / wrong device";
    case KSDF_ERR_UNSUPPORTED: return "unsupported";
    case KSDF_ERR_OUT_OF_MEMORY: return "out of device memory";
    case KSDF_ERR_TIMEOUT: return "a bounded wait expired";
    default: return "unknown status";
  }
}

extern "C" const char* ksdf_last_error(void) { return g_last_error.c_str(); }
