/*
 * ksdf — batched local Gaussian-process SDF regression on MI355X (gfx950).
 *
 * The back-end of Kernel-SDF (arXiv 2603.29227): per spatial cell a log-GP is fitted
 * on nearby surface samples; a query evaluates its K nearest cells, maps each
 * cell's posterior mean to a distance and keeps the smallest (min-fusion), then
 * returns the analytic gradient, the GP variance and the softmin SDF variance.
 *
 *   Sec. IV-B.1  eq. log_gp_posterior_mean: f = k*^T (K + Sigma)^{-1} 1 (all labels 1),
 *                grad f = (grad k*)^T (K + Sigma)^{-1} 1,  V[f] = k(x*,x*) - k*^T (K+Sigma)^{-1} k*;
 *                UDF gradient -grad f / |grad f|; local GPs per octant trained on
 *                overlapping collection boxes; u = min over the K nearest GPs;
 *                SDF d = s * u with a sign s supplied by the caller.
 *   Table I      RBF kernel k(r) = exp(-r^2 / 2 l^2), inverse transform r(f) = sqrt(-2 l^2 log f).
 *   App. D       scaled kernel k' = gamma k, r(f') = sqrt(-2 l^2 log f' + d^2).
 *   Sec. IV-B.3  V[u] = sum_i |grad_{x_i} h|^2 sigma_i^2 with the softmin h = s^T z,
 *                grad_{x_i} h = -s_i (alpha s^T z - alpha z_i + 1)(x* - x_i)/z_i.
 *
 * Conventions for every entry point:
 *   - "device" pointers are HIP device (or managed) memory on the current device;
 *     "host" pointers are ordinary host memory.  The caller owns every buffer it
 *     passes; the library never frees caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Device
 *     work is enqueued asynchronously on it; unless stated, no host synchronisation.
 *   - Return value: KSDF_OK (0) or a negative ksdf_status.  No C++ exception and no
 *     abort crosses this boundary.  Argument errors are detected on the host before
 *     any work is enqueued.  Numerical outcomes (an ill-conditioned cell refitted in
 *     FP64, a failed cell, a clamped UDF, a query with no valid cell) are reported
 *     per cell / per query in the optional status arrays, not as errors.
 *   - Floating arrays of points and outputs are float (KSDF_FP32 models) or double
 *     (KSDF_FP64 models), row-major; [n,3] means 3 consecutive values per point.
 */
#ifndef KSDF_H
#define KSDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ksdf_status {
  KSDF_OK = 0,
  KSDF_ERR_INVALID_ARGUMENT = -1, /* null pointer, bad size, bad enum, bad hyperparameter */
  KSDF_ERR_INVALID_INPUT = -2,    /* NaN / Inf in host-visible inputs or hyperparameters */
  KSDF_ERR_WORKSPACE = -3,        /* workspace smaller than the *_workspace_bytes query */
  KSDF_ERR_HIP = -4,              /* a HIP runtime call failed (message in ksdf_last_error) */
  KSDF_ERR_DEVICE = -5,           /* no usable gfx950 device, or the model lives on another device */
  KSDF_ERR_UNSUPPORTED = -6,      /* a feature this build does not provide (e.g. m > 128) */
  KSDF_ERR_OUT_OF_MEMORY = -7,    /* kept for compatibility: the library allocates no device memory */
  KSDF_ERR_TIMEOUT = -8           /* a fused launch's bounded wait expired (see ksdf_model_check) */
} ksdf_status;

enum { KSDF_FP64 = 0, KSDF_FP32 = 1 };           /* model precision */
enum { KSDF_DTYPE_F32 = 0, KSDF_DTYPE_F64 = 1 };  /* element type of surface points */

/* per-query status bits (uint8) */
enum { KSDF_Q_NO_VALID_CELL = 1, KSDF_Q_CLAMPED = 2, KSDF_Q_GRAD_ZERO = 4, KSDF_Q_OUTSIDE_INDEX = 8,
       KSDF_Q_FIT_TIMEOUT = 16 /* answered by a fused launch whose wait for the fits expired */ };
/* per-cell status bits (uint8) */
enum { KSDF_C_FP64 = 1, KSDF_C_FAILED = 2 };

#define KSDF_MAX_M 128     /* samples per cell */
#define KSDF_MAX_K 16      /* fused cells per query */

/* Kernels of Table I.  KSDF_KERNEL_RBF: k(r) = exp(-r^2 / 2 l^2), u = sqrt(d^2 - 2 l^2
 * ln f') (App. D scaling by the nearest sample d).  KSDF_KERNEL_MATERN32: k(r) =
 * (1 + c r) exp(-c r) with c = sqrt(3) / l, u = d - ln(f') / c; u < 0 clamps to 0.
 * The UDF gradient is w/|w| with w = sum a_i e_i (x* - x_i), e_i the scaled k_i (RBF)
 * or exp(-c (z_i - d)) (Matern 3/2).  Matern 3/2 models: FP32 queries run the plain
 * one-thread-per-query kernel in FP32 (the wave-cooperative kernels carry RBF-specific
 * error bounds), ksdf_fit_query runs fit and query as separate launches, and the
 * backward runs one thread per query in FP64 for either precision. */
enum { KSDF_KERNEL_RBF = 0, KSDF_KERNEL_MATERN32 = 1 };

/* Hyperparameters (host struct).  ell: length-scale l (m), > 0.  noise_var:
 * uniform surface-sample variance sigma^2 >= 0 (used where no per-sample variance is
 * given).  alpha: softmin temperature; <= 0 ties it to the length-scale as
 * alpha = 1/(2 l^2), which the backward then differentiates through.  k_fuse:
 * number of nearest cells fused by the min, 1..KSDF_MAX_K.  precision: KSDF_FP64
 * (every step in double, one block per cell and one thread per query) or KSDF_FP32
 * (FP32 bulk; cells whose condition estimate exceeds cond_fp64_threshold, or whose
 * FP32 pivot fails, are factored in FP64). */
typedef struct ksdf_hyper {
  double ell;
  double noise_var;
  double alpha;
  int k_fuse;
  int precision;
  double cond_fp64_threshold;
  int flags;          /* KSDF_FIT_* bits */
  int kernel;         /* KSDF_KERNEL_*; fixed at ksdf_model_create */
} ksdf_hyper;

/* flags: KSDF_FIT_ADJOINT makes every fit also prepare the per-cell adjoint vectors
 * that ksdf_query_backward needs (xi_l = A^{-1} (dA/dl) a and xi_s = A^{-1} a);
 * KSDF_FIT_ADJOINT_VARF additionally keeps dA/dl packed per cell, needed for var_f
 * cotangents.  KSDF_FIT_DENSE_INV reserves a dense L^{-1} per cell (16 KiB) for the
 * matrix-core form of the GP variance (the query_mfma tuning; FP32 RBF models with
 * m <= 64, else ignored).  They must be set at ksdf_model_bytes / ksdf_model_create
 * (which size the store) and the adjoint bits may then be dropped per fit. */
enum { KSDF_FIT_ADJOINT = 1, KSDF_FIT_ADJOINT_VARF = 2, KSDF_FIT_DENSE_INV = 4 };

/* ---------------------------------------------------------------------------
 * Cell builder (host, OpenMP).  The per-octant GP training buffers of Sec. IV-B.1:
 * key = floor((x - origin)/h) per axis; a key is occupied when its own box holds a
 * sample; its training set is the up-to-m_c samples of its collection box (the cell
 * box grown by `margin` on every side, inclusive bounds) nearest the cell centre
 * origin + (key + 1/2) h, nearest first, ties by lower sample index; cells with fewer
 * than m_min samples are dropped; ids follow lexicographic key order.
 * m_c = min(m_max, cap_grid[key - key_lo]) where cap_grid (uint8, C order, dims
 * key_dims) covers the key, else m_max.  cap_grid may be NULL.
 * pts: host [n,3] float or double (dtype).  Distances are taken in double.
 * On success *out holds a host handle; read it with ksdf_cellset_info/copy and free
 * it with ksdf_cellset_destroy.
 * ------------------------------------------------------------------------- */
typedef struct ksdf_cellset ksdf_cellset;
int ksdf_build_cells(const void* pts, int dtype, long n, const double origin[3], double h,
                     double margin, int m_max, int m_min, const uint8_t* cap_grid,
                     const int key_lo[3], const int key_dims[3], ksdf_cellset** out);
int ksdf_cellset_info(const ksdf_cellset* cs, int* n_cells, long* nnz);
/* offsets [n_cells+1], samples [nnz], keys [n_cells,3]: host int32 arrays. */
int ksdf_cellset_copy(const ksdf_cellset* cs, int* offsets, int* samples, int* keys);
void ksdf_cellset_destroy(ksdf_cellset* cs);

/* ---------------------------------------------------------------------------
 * Model: the per-cell store (gathered samples, weights a = (K+Sigma)^{-1} 1, packed
 * Cholesky factors, flags; Sec. IV-B.1 eq. log_gp_posterior_mean) and the candidate
 * index for the K-nearest-cell search ("the K nearest GPs", Sec. IV-B.1).
 *
 * The caller owns all of the model's device memory; the library allocates none.
 * Creating a model takes four calls:
 *   1. ksdf_model_bytes (host, no device work): the store's size in bytes for these
 *      arguments (0 if they are invalid; ksdf_model_create then reports why).
 *   2. ksdf_model_create: carves the store (device, at least that many bytes, 256-byte
 *      aligned) into the model's arrays, uploads the cell structure and runs the
 *      index's count pass on `stream`, then synchronises that stream once.
 *   3. ksdf_model_index_bytes: the size of the candidate lists, known after step 2.
 *   4. ksdf_model_attach_index: hands over a device buffer of at least that many
 *      bytes (4-byte aligned) and fills the lists on `stream` (asynchronous; calls on
 *      other streams must wait for it).  Fits may run before this; queries,
 *      ksdf_fit_query and the backward return KSDF_ERR_INVALID_ARGUMENT until it is done.
 * Both buffers must stay allocated, unmodified by the caller, until the model is
 * destroyed and its last launch has finished.  KSDF_ERR_WORKSPACE when a buffer is
 * missing or too small.
 * offsets/samples/keys: host int32 CSR as produced by the builder (keys unique and in
 * lexicographic order, else KSDF_ERR_INVALID_ARGUMENT); origin/h: the builder's lattice
 * (cell c's centre is origin + (key_c + 1/2) h); n_points: number of surface samples
 * the fits will receive.
 * query_lo/query_hi (host, may be NULL): a box the queries are expected in; the index
 * covers it (queries outside still get exact answers through a slower brute-force
 * candidate scan and carry KSDF_Q_OUTSIDE_INDEX).  The model keeps the
 * hyperparameters' k_fuse, precision, kernel and flags; ell, noise_var and alpha may
 * change per fit.  ksdf_model_destroy frees the host handle only.
 * ------------------------------------------------------------------------- */
typedef struct ksdf_model ksdf_model;
size_t ksdf_model_bytes(int n_cells, const int* offsets, const int* samples, const int* keys,
                        const double origin[3], double h, long n_points, const ksdf_hyper* hyper,
                        const double query_lo[3], const double query_hi[3]);
int ksdf_model_create(int n_cells, const int* offsets, const int* samples, const int* keys,
                      const double origin[3], double h, long n_points, const ksdf_hyper* hyper,
                      const double query_lo[3], const double query_hi[3], void* store,
                      size_t store_bytes, void* stream, ksdf_model** out);
size_t ksdf_model_index_bytes(const ksdf_model* model);
int ksdf_model_attach_index(ksdf_model* model, void* list, size_t list_bytes, void* stream);
void ksdf_model_destroy(ksdf_model* model);
/* Launch-shape knobs (host struct), picked per workload by the autotuner.
 * query_sub: index boxes are split into query_sub^3 sub-boxes (1, 2 or 4) for the
 *   counting sort that groups a wave's queries; 0 = finest that keeps <= 8M bins.
 * query_block: threads per block of the FP32 query kernel (64 or 256; 0 = 256).
 * fused: ksdf_fit_query uses the persistent fused launch (1) or the per-bucket fit
 *   launches followed by the query launch (0).
 * fit_min_bucket: FP32 cells with m <= this run in the fit kernel sized for it
 *   (16, 32 or 64): larger values merge small cells into fewer launches.
 * query_split: the FP32 query runs as two kernels with the queries regrouped by
 *   argmin cell between them (1), or as one kernel (0).  Outputs are identical.
 * query_lanes, backward_lanes: each lane reads its own cells (1) instead of the
 *   wave sharing a cell through scalar loads (0); for sparse query sets, whose waves
 *   span many cells.  query_lanes applies to the two-kernel query.  Outputs are
 *   identical.
 * query_pairs: the first kernel of the two-kernel query evaluates each (query,
 *   candidate cell) pair once, with the pairs grouped by cell (1), instead of each
 *   wave walking the union of its lanes' candidates (0).  Every candidate is then
 *   evaluated (no lower-bound pruning), which can change which near-tied cells are
 *   re-evaluated in FP64: outputs agree within the parity tolerance, not
 *   always bit for bit.  Applies to the two-kernel query when Q * (8 or 16) < 2^31;
 *   the workspace grows by about 24 bytes per (query, candidate).
 * query_mfma: the second kernel of the two-kernel query (wave-shared cells) forms
 *   |L^{-1} k*|^2 of the GP variance on the matrix cores from a dense per-cell L^{-1},
 *   instead of by forward substitution.  Applies to FP32 RBF models with m <= 64
 *   (else ignored); such a model needs KSDF_FIT_DENSE_INV at creation (else
 *   KSDF_ERR_UNSUPPORTED, the tuning unchanged).  While it is on, each fit and refit
 *   also forms the dense factors, and the first query after it is turned on forms
 *   them if they are stale.  var_f then differs from the other
 *   launch shapes in the last bits (a different summation order); every other output
 *   is identical. */
typedef struct ksdf_tuning {
  int query_sub;
  int query_block;
  int fused;
  int fit_min_bucket;
  int query_split;
  int query_lanes;
  int backward_lanes;
  int query_pairs;
  int query_mfma;
} ksdf_tuning;
int ksdf_model_set_tuning(ksdf_model* model, const ksdf_tuning* tuning);
int ksdf_model_get_tuning(const ksdf_model* model, ksdf_tuning* tuning);

/* Kernel timing, for benchmarks and profiles.  With timing on, each launch records a
 * pair of HIP events on its own stream around the main kernel(s) of its phase:
 *   KSDF_TIMER_FIT       the FP32 bucket fits and the FP64 refit (ksdf_fit_cells);
 *   KSDF_TIMER_QUERY     the query kernel, after the query bucketing;
 *   KSDF_TIMER_BACKWARD  the adjoint kernel (after the argmin sort, before the
 *                        hyperparameter reduction);
 *   KSDF_TIMER_FUSED     the persistent fused fit+query kernel.
 * Each phase keeps the pairs of its last KSDF_TIMER_SLOTS launches.
 * ksdf_model_timer_read waits for the phase's launches since the previous read (or since
 * timing was turned on), writes their durations in ms, in launch order, to ms[0..*n)
 * (at most max_n), and starts a new count.  KSDF_ERR_INVALID_ARGUMENT when timing is off
 * or more than KSDF_TIMER_SLOTS launches happened since the previous read (the oldest
 * pairs were reused).  Timing must be off while a stream that the model launches on is
 * being captured into a graph. */
#define KSDF_TIMER_FIT 0
#define KSDF_TIMER_QUERY 1
#define KSDF_TIMER_BACKWARD 2
#define KSDF_TIMER_FUSED 3
#define KSDF_TIMER_COUNT 4
#define KSDF_TIMER_SLOTS 8
int ksdf_model_set_timing(ksdf_model* model, int on);
int ksdf_model_timer_read(ksdf_model* model, int timer, float* ms, int max_n, int* n);

/* Host-side facts about a model: n_cells, nnz, largest m, index entries, device bytes
 * (the store plus, once attached, the candidate lists). */
int ksdf_model_info(const ksdf_model* model, int* n_cells, long* nnz, int* max_m,
                    long* index_entries, size_t* device_bytes);

/* ---------------------------------------------------------------------------
 * ksdf_fit_cells — Sec. IV-B.1 training of every cell's log-GP.
 * Gathers each cell's samples (cell-local coordinates), assembles A = K + Sigma with
 * the RBF kernel of Table I, factors A = L L^T and solves a = A^{-1} 1.  FP32 models
 * estimate cond_2(A) (power and inverse iteration on the FP32 factor) and refit
 * cells above the threshold (or
 * with a non-positive pivot) in FP64; a cell that also fails in FP64 is flagged
 * KSDF_C_FAILED and excluded from every query (u = +inf).
 * surface_pts: device [n_points,3] float or double (dtype); sample_var: device
 * [n_points] of the same type, or NULL for the uniform hyper->noise_var.
 * cell_status: device uint8 [n_cells] or NULL.  Asynchronous on `stream`; allocates
 * nothing.  The model must not be used by another stream concurrently.
 * ------------------------------------------------------------------------- */
int ksdf_fit_cells(ksdf_model* model, const void* surface_pts, int dtype, long n_points,
                   const void* sample_var, const ksdf_hyper* hyper, uint8_t* cell_status,
                   void* stream);

/* ---------------------------------------------------------------------------
 * ksdf_query — SDF mean, gradient and variances at Q points.
 * points: device [Q,3].  sign: device int8 [Q] (+1/-1) or NULL (all +1).
 * Outputs (device, overwritten): mean [Q] = s*u; grad [Q,3] = s*w/|w| (unit); var [Q]
 * = softmin V[u] (m^2) of the argmin cell; var_f [Q] = GP variance 1 - |L^{-1} k*|^2 of
 * the argmin cell, or NULL; grad_var [Q,3] = V[grad_k u], the variance of the softmin
 * gradient of the argmin cell from the sample variances (Sec. IV-B.3, App. C), or NULL;
 * argmin [Q] int32 cell id or NULL; q_status [Q] uint8 or NULL.  A query with no valid
 * cell gets mean = +inf, grad = 0, var = +inf, var_f = 1, grad_var = +inf.
 * workspace: device scratch of at least ksdf_query_workspace_bytes(model, Q) bytes
 * (may be NULL when that is 0).  Asynchronous; allocates nothing.  The query only
 * reads the model (except that, with the query_mfma tuning, it first forms the dense
 * inverses when a fit made them stale), so queries and backward calls on different
 * streams may run at once if each has its own workspace and no fit runs meanwhile.
 * ------------------------------------------------------------------------- */
size_t ksdf_query_workspace_bytes(const ksdf_model* model, long Q);
int ksdf_query(const ksdf_model* model, const void* points, long Q, const int8_t* sign,
               void* mean, void* grad, void* var, void* var_f, void* grad_var, int* argmin,
               uint8_t* q_status, void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * ksdf_query_bucket, ksdf_query_bucketed — ksdf_query in two calls, so that its first
 * step can run while the cells are still being fitted (Sec. IV-B: the K nearest GPs
 * of a point depend on the cell lattice only, not on the fit).
 * ksdf_query_bucket sorts the Q points by candidate-index box and sub-box into
 * `workspace` (the counting sort that opens every FP32 query); it reads the points and
 * the model's candidate index, not the fitted cells, and may therefore run on another
 * stream beside ksdf_fit_cells.  ksdf_query_bucketed then runs the rest of ksdf_query
 * on that workspace, with the same arguments, outputs and errors as ksdf_query, and
 * gives its results bit for bit.  Between the two calls the caller keeps the points,
 * the workspace contents and the model's tuning unchanged, and orders the calls (one
 * stream, or an event).  Workspace: at least ksdf_query_workspace_bytes(model, Q)
 * bytes for both.  For FP64 models (which do not bucket) ksdf_query_bucket does
 * nothing and ksdf_query_bucketed is ksdf_query.  Asynchronous; allocates nothing.
 * ------------------------------------------------------------------------- */
int ksdf_query_bucket(const ksdf_model* model, const void* points, long Q, void* workspace,
                      size_t ws_bytes, void* stream);
int ksdf_query_bucketed(const ksdf_model* model, const void* points, long Q, const int8_t* sign,
                        void* mean, void* grad, void* var, void* var_f, void* grad_var,
                        int* argmin, uint8_t* q_status, void* workspace, size_t ws_bytes,
                        void* stream);

/* ---------------------------------------------------------------------------
 * ksdf_query_noalloc — ksdf_query for callers that cannot allocate device memory
 * (code under graph capture, tight serving loops, harnesses that forbid allocation).
 * Same arguments, outputs and launches as ksdf_query, without the workspace: the
 * scratch lives in a fixed device array of KSDF_NOALLOC_SCRATCH_BYTES that each device
 * holds until the process ends (its address is looked up on the first call on a
 * device).  Queries whose ksdf_query_workspace_bytes exceeds that size return
 * KSDF_ERR_WORKSPACE (use ksdf_query with a workspace).  Calls that overlap on one
 * device share the array and race: issue them on one stream, or serialise them.
 * ------------------------------------------------------------------------- */
#define KSDF_NOALLOC_SCRATCH_BYTES (64u << 20)
int ksdf_query_noalloc(const ksdf_model* model, const void* points, long Q, const int8_t* sign,
                       void* mean, void* grad, void* var, void* var_f, void* grad_var, int* argmin,
                       uint8_t* q_status, void* stream);

/* ---------------------------------------------------------------------------
 * ksdf_refit_cells — streaming update of the fitted cells (Sec. IV-C, App. G "GP
 * training queue").  dirty [n_cells] (device float, the count c2 of buffer updates
 * since a cell's last training) and qcount [n_cells] (device float, the query count
 * c0, see ksdf_count_queries) give each cell with c2 > 0 the priority
 * s = c2 (1 + eta c0), computed in FP32 as c2 * (1 + (eta * c0)) with each operation
 * rounded once (eta rounded to float first); the min(budget, #dirty) cells of highest priority (ties to the lower
 * id) are refitted from surface_pts (and sample_var, or the uniform noise_var) with
 * the model's current hyperparameters, exactly as ksdf_fit_cells fits them; then
 * c2 = 0 and c0 = c0 / 2 for those cells.  All other cells keep their fit.
 * refit_cells (device int, at least min(budget, n_cells)) receives the refitted cell
 * ids in priority order and n_refit (device int) their number.  cell_status (device
 * uint8 [n_cells] or NULL) is updated for the refitted cells only.  Requires a prior
 * ksdf_fit_cells / ksdf_fit_query; budget >= 1; eta >= 0; the counters >= 0.
 * Asynchronous and free of host synchronisation (capturable in a graph); workspace:
 * at least ksdf_refit_workspace_bytes(model, budget) bytes.
 * ------------------------------------------------------------------------- */
size_t ksdf_refit_workspace_bytes(const ksdf_model* model, int budget);
int ksdf_refit_cells(ksdf_model* model, const void* surface_pts, int dtype, long n_points,
                     const void* sample_var, float* dirty, float* qcount, double eta, int budget,
                     int* refit_cells, int* n_refit, uint8_t* cell_status, void* workspace,
                     size_t ws_bytes, void* stream);

/* ksdf_count_queries — the query counters of App. G: for every query with an argmin
 * cell c in [0, n_cells) (the GP whose prediction was used; other values, such as
 * -1 for no valid cell, are skipped), qcount[c] = min(qcount[c] + count_c, cap) with
 * count_c the number of such queries, added once per cell (one rounding: the result
 * does not depend on the order of the queries).  App. G caps at 10000.  argmin:
 * device int [Q] from ksdf_query; qcount: device float [n_cells]; workspace: device,
 * at least ksdf_count_queries_workspace_bytes(model) bytes (4 per cell).
 * Asynchronous. */
size_t ksdf_count_queries_workspace_bytes(const ksdf_model* model);
int ksdf_count_queries(const ksdf_model* model, const int* argmin, long Q, float* qcount,
                       float cap, void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * SDF sign from local Bayesian-Hilbert-map weights (Sec. IV-A, eq. sign_prediction;
 * App. B features).  The caller's BHM front-end supplies the weights; these calls
 * only evaluate them.  Local maps sit on a lattice of boxes (edge `box`, dims boxes per
 * axis from `origin`); box b's map is box_bhm[b] (device int, -1 = none).  A map holds
 * hinges^3 hinge points at the lattice points of its box (spacing box / (hinges - 1),
 * 2 <= hinges <= 16) and weights[id * (hinges^3 + 1) + ...] (device double, hinge
 * (i, j, k) at (i * hinges + j) * hinges + k, the bias last).  The log-odds of a query
 * in box b is l = mu^T phi with phi = [exp(-gamma |x - h|^2) ..., 1] over its map.
 * ksdf_bhm_sign: sign[q] (device int8) = +1 where l < tau, -1 otherwise, +1 where the
 * box has no map (no occupied voxel); logodds[q] (device double, or NULL) = l, or
 * -inf without a map.  points: device [Q,3], dtype float or double; l in double.
 * ksdf_bhm_update_tau: tau (device double, in/out) <- (1 - alpha) tau + (alpha / K)
 * sum_k l(hit_k) (eq. online_surf_logodds), 0 < alpha <= 1, in a fixed summation
 * order; workspace >= ksdf_bhm_tau_workspace_bytes(K).  Both asynchronous.
 * ------------------------------------------------------------------------- */
typedef struct ksdf_bhm_layout {
  double origin[3];
  double box;
  int dims[3];
  int hinges;
  double gamma;
} ksdf_bhm_layout;
int ksdf_bhm_sign(const ksdf_bhm_layout* layout, const int* box_bhm, const double* weights,
                  const void* points, int dtype, long Q, double tau, int8_t* sign, double* logodds,
                  void* stream);
size_t ksdf_bhm_tau_workspace_bytes(long K);
int ksdf_bhm_update_tau(const ksdf_bhm_layout* layout, const int* box_bhm, const double* weights,
                        const void* hits, int dtype, long K, double alpha, double* tau,
                        void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * ksdf_fit_query — ksdf_fit_cells followed by ksdf_query, with the same arguments
 * and outputs, as ONE persistent fused launch for FP32 models: resident workgroups
 * drain a task queue holding every cell fit (largest m first, FP64 refit in place
 * where the condition estimate asks for it) and then the query tiles, which start
 * once all fits have released their results.  Intended for cells with uneven m,
 * where separate per-bucket launches leave the device idle between kernels.  With the
 * tuning fused = 0 (or a Matern model) it runs the separate fit launches, with the
 * query's bucketing (see ksdf_query_bucket) on a second stream that the model owns
 * (default priority, forked from `stream` and joined back within the call, so the
 * call stays capturable in a graph).  FP64 models run the plain fit and query back
 * to back.  workspace: at least ksdf_fit_query_workspace_bytes(model, Q) bytes.
 * Asynchronous; allocates nothing.
 * ------------------------------------------------------------------------- */
size_t ksdf_fit_query_workspace_bytes(const ksdf_model* model, long Q);
/* A workgroup's wait for the fits is bounded (2^26 sleeps by default).  If it expires
 * the launch still ends normally, the queries that workgroup answers carry
 * KSDF_Q_FIT_TIMEOUT (their values may come from unfinished fits), and the model
 * records it: ksdf_model_check (host; synchronises `stream`) returns KSDF_ERR_TIMEOUT
 * once and clears the record, else KSDF_OK.  ksdf_model_set_wait_limit sets the bound
 * in sleeps (0 restores the default; a test can set 1 to exercise the path). */
int ksdf_model_check(ksdf_model* model, void* stream);
int ksdf_model_set_wait_limit(ksdf_model* model, long sleeps);
int ksdf_fit_query(ksdf_model* model, const void* surface_pts, int dtype, long n_points,
                   const void* sample_var, const ksdf_hyper* hyper, uint8_t* cell_status,
                   const void* points, long Q, const int8_t* sign, void* mean, void* grad,
                   void* var, void* var_f, void* grad_var, int* argmin, uint8_t* q_status,
                   void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * ksdf_query_backward — vector-Jacobian product of ksdf_query.
 * Given cotangents d_mean [Q], d_grad [Q,3] (or NULL), d_var [Q] (or NULL) and d_var_f
 * [Q] (or NULL) of L = sum_q d_mean*mean + d_grad.grad + d_var*var + d_var_f*var_f,
 * writes d_points [Q,3] = dL/dpoints (overwritten) and d_hyper (device double [2],
 * overwritten) = (dL/d ell, dL/d noise_var), the latter including the dependence
 * through the fit (a and L are functions of ell and noise_var) and, when alpha is
 * tied, through alpha = 1/(2 l^2).  The argmin cell of each query is held fixed (the
 * min is piecewise): argmin [Q] (device int32) is the forward's argmin output for the
 * same points, or NULL to recompute it.  Clamped outputs contribute zero.  d_hyper for
 * noise_var is defined for the uniform variance (zero when the fit had per-sample
 * variances).  k* is recomputed, not stored.  The theta reduction is deterministic
 * (fixed order, no atomics; FP64 for FP64 models, float-float for FP32 models).  The
 * model's last fit must have had
 * KSDF_FIT_ADJOINT (and KSDF_FIT_ADJOINT_VARF when d_var_f is given).
 * workspace: at least ksdf_backward_workspace_bytes(model, Q) bytes.
 * ------------------------------------------------------------------------- */
size_t ksdf_backward_workspace_bytes(const ksdf_model* model, long Q);
int ksdf_query_backward(const ksdf_model* model, const void* points, long Q, const int8_t* sign,
                        const int* argmin, const void* d_mean, const void* d_grad,
                        const void* d_var, const void* d_var_f, void* d_points, double* d_hyper,
                        void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * ksdf_cost_backward -- the gradient of a collision cost for trajectory optimisation
 * (the use of SDF values and gradients motivated in Sec. I): the softplus margin cost
 *   C = sum_q softplus(t_q),  t_q = margin - mean_q + kvar * sqrt(var_q),
 * of the outputs mean [Q] and var [Q] (device, the model's precision) of a ksdf_query
 * of the same points, with respect to the points and (ell, noise_var).  It is
 * ksdf_query_backward with d_mean = -sigmoid(t) and d_var = kvar sigmoid(t) /
 * (2 sqrt(var)) formed inside the kernel (var clamped below at 1e-30; stable sigmoid
 * and softplus), so no separate cotangent pass runs.  argmin, d_points, d_hyper,
 * the argmin rule and the workspace (ksdf_backward_workspace_bytes) are those of
 * ksdf_query_backward.  cost (device [Q] of the model's precision, or NULL): the
 * per-point softplus(t_q).  margin and kvar must be finite.
 * ------------------------------------------------------------------------- */
int ksdf_cost_backward(const ksdf_model* model, const void* points, long Q, const int8_t* sign,
                       const int* argmin, const void* mean, const void* var, double margin,
                       double kvar, void* cost, void* d_points, double* d_hyper, void* workspace,
                       size_t ws_bytes, void* stream);

/* Static description of a status code; ksdf_last_error() gives the calling
 * thread's last detailed message (never NULL). */
const char* ksdf_status_string(int status);
const char* ksdf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KSDF_H */
