// FP64 CPU oracle for the local-GP SDF back-end of Kernel-SDF (arXiv 2603.29227).
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  It shares no code with
// the HIP path and must never serve as a fallback for it.
//
// Plain, slow, obviously correct: every step follows the paper's definitions in
// their own order, in double precision, with straightforward loops and no
// blocking or fusion.  Sections cited below are the paper's:
//   Sec. IV-B.1  log-GP posterior mean, gradient and variance (eq. log_gp_posterior_mean),
//                kernel vector / matrix / noise, UDF gradient, local GPs per octant with
//                overlapping collection boxes, min-fusion of the K nearest GPs
//   Table I      RBF and Matern 3/2 kernels and their inverse transforms r(f)
//   App. D       adaptive scaling (RBF: gamma = exp(d^2 / 2 l^2), r(f') = sqrt(-2 l^2 log f' + d^2);
//                Matern 3/2: gamma = exp(sqrt(3) d / l), r(f') = -(l / sqrt(3)) log f' + d)
//   Sec. IV-B.3  softmin SDF variance V[u] = sum_i |grad_{x_i} h|^2 sigma_i^2
//   Sec. IV-B.1  sign decomposition d = s * u
//
// Readings where the paper is silent (all shared with the GPU path as inputs):
//   cells: collection box = cell box grown by `margin` per side; up to m_c samples
//   nearest the cell centre (ties by lower sample index); candidate GPs = the
//   K nearest occupied cell centres (ties by id); d in App. D = nearest sample;
//   f' <= 0 excludes the cell (u = +inf); u^2 < 0 (RBF) or u < 0 (Matern) clamps
//   u to 0; softmin temperature alpha = 1/(2 l^2) unless given, for both kernels.
//
// Scalar type T is double for the forward pass and Dual<N> (forward-mode
// automatic differentiation) for the vector-Jacobian products.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <tuple>
#include <vector>

#include <omp.h>

namespace {

// ---------------------------------------------------------------------------
// forward-mode dual numbers
// ---------------------------------------------------------------------------
template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0) { for (int k = 0; k < N; ++k) d[k] = 0; }
  Dual(double x) : v(x) { for (int k = 0; k < N; ++k) d[k] = 0; }  // NOLINT
};
template <int N> Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v + b.v); for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v - b.v); for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r(-a.v); for (int k = 0; k < N; ++k) r.d[k] = -a.d[k]; return r; }
template <int N> Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v * b.v); for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
template <int N> Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v / b.v);
  for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r; }
template <int N> Dual<N> exp(const Dual<N>& a) {
  Dual<N> r(std::exp(a.v)); for (int k = 0; k < N; ++k) r.d[k] = r.v * a.d[k]; return r; }
template <int N> Dual<N> log(const Dual<N>& a) {
  Dual<N> r(std::log(a.v)); for (int k = 0; k < N; ++k) r.d[k] = a.d[k] / a.v; return r; }
template <int N> Dual<N> sqrt(const Dual<N>& a) {
  Dual<N> r(std::sqrt(a.v));
  for (int k = 0; k < N; ++k) r.d[k] = (r.v > 0) ? a.d[k] / (2 * r.v) : 0.0;
  return r; }
template <int N> Dual<N> log1p(const Dual<N>& a) {
  Dual<N> r(std::log1p(a.v)); for (int k = 0; k < N; ++k) r.d[k] = a.d[k] / (1 + a.v); return r; }
template <int N> Dual<N> fabs(const Dual<N>& a) { return a.v < 0 ? -a : a; }

inline double val(double x) { return x; }
template <int N> double val(const Dual<N>& x) { return x.v; }

using std::exp; using std::log; using std::sqrt; using std::log1p; using std::fabs;

// ---------------------------------------------------------------------------
// cells (the per-octant GP training buffers with overlapping collection boxes)
// ---------------------------------------------------------------------------
struct Key { long i, j, k; };
bool operator<(const Key& a, const Key& b) {
  return std::tie(a.i, a.j, a.k) < std::tie(b.i, b.j, b.k);
}

struct CellSet {
  std::vector<int> offsets, samples, keys;
  std::vector<double> centres;
};

}  // namespace

extern "C" {

// Build the cells.  Keys are floor((x - origin) / h) per axis; a key is occupied
// when its own box holds a sample; its training set is the up-to-m_c samples of
// the collection box (cell box grown by `margin`, bounds inclusive) nearest the
// cell centre origin + (key + 1/2) h, ties by lower sample index; cells with fewer
// than m_min samples are dropped; ids follow lexicographic key order.
void* oracle_cells_build(const double* pts, long n, const double* origin, double h,
                         double margin, int m_max, int m_min, const uint8_t* cap_grid,
                         const int* key_lo, const int* key_dims) {
  std::map<Key, std::vector<long>> bins;
  for (long s = 0; s < n; ++s) {
    Key k{(long)std::floor((pts[3 * s + 0] - origin[0]) / h),
          (long)std::floor((pts[3 * s + 1] - origin[1]) / h),
          (long)std::floor((pts[3 * s + 2] - origin[2]) / h)};
    bins[k].push_back(s);
  }
  const long reach = (long)std::ceil(margin / h) + 1;
  auto* out = new CellSet;
  out->offsets.push_back(0);
  for (const auto& kv : bins) {
    const Key& c = kv.first;
    double lo[3], hi[3], ctr[3];
    const long kc[3] = {c.i, c.j, c.k};
    for (int d = 0; d < 3; ++d) {
      lo[d] = origin[d] + (double)kc[d] * h - margin;
      hi[d] = origin[d] + (double)(kc[d] + 1) * h + margin;
      ctr[d] = origin[d] + ((double)kc[d] + 0.5) * h;
    }
    std::vector<std::pair<double, long>> cand;
    for (long di = -reach; di <= reach; ++di)
      for (long dj = -reach; dj <= reach; ++dj)
        for (long dk = -reach; dk <= reach; ++dk) {
          auto it = bins.find(Key{c.i + di, c.j + dj, c.k + dk});
          if (it == bins.end()) continue;
          for (long s : it->second) {
            const double* x = pts + 3 * s;
            bool in = true;
            for (int d = 0; d < 3; ++d) in = in && (x[d] >= lo[d]) && (x[d] <= hi[d]);
            if (!in) continue;
            double dx = x[0] - ctr[0], dy = x[1] - ctr[1], dz = x[2] - ctr[2];
            double r2 = dx * dx + dy * dy + dz * dz;
            cand.push_back({r2, s});
          }
        }
    std::sort(cand.begin(), cand.end());
    long m_c = m_max;
    if (cap_grid) {
      long g[3] = {kc[0] - key_lo[0], kc[1] - key_lo[1], kc[2] - key_lo[2]};
      if (g[0] >= 0 && g[0] < key_dims[0] && g[1] >= 0 && g[1] < key_dims[1] && g[2] >= 0 &&
          g[2] < key_dims[2])
        m_c = std::min<long>(m_max, cap_grid[(g[0] * key_dims[1] + g[1]) * key_dims[2] + g[2]]);
    }
    long take = std::min<long>(m_c, (long)cand.size());
    if (take < m_min) continue;
    for (long t = 0; t < take; ++t) out->samples.push_back((int)cand[t].second);
    out->offsets.push_back((int)out->samples.size());
    out->keys.push_back((int)c.i); out->keys.push_back((int)c.j); out->keys.push_back((int)c.k);
    for (int d = 0; d < 3; ++d) out->centres.push_back(ctr[d]);
  }
  return out;
}

int oracle_cells_count(void* hdl, long* nnz) {
  auto* c = static_cast<CellSet*>(hdl);
  *nnz = (long)c->samples.size();
  return (int)c->offsets.size() - 1;
}

void oracle_cells_copy(void* hdl, int* offsets, int* samples, int* keys, double* centres) {
  auto* c = static_cast<CellSet*>(hdl);
  std::copy(c->offsets.begin(), c->offsets.end(), offsets);
  std::copy(c->samples.begin(), c->samples.end(), samples);
  std::copy(c->keys.begin(), c->keys.end(), keys);
  std::copy(c->centres.begin(), c->centres.end(), centres);
}

void oracle_cells_free(void* hdl) { delete static_cast<CellSet*>(hdl); }

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// kernels of Table I as functions of the squared distance
// ---------------------------------------------------------------------------
enum { KERNEL_RBF = 0, KERNEL_MATERN32 = 1 };

// Matern 3/2 rate c = sqrt(3) / l: k(r) = (1 + c r) exp(-c r).
template <class T>
T matern_rate(const T& ell) { return T(std::sqrt(3.0)) / ell; }

// k(r) from r^2.  RBF: exp(-r^2 / 2 l^2); Matern 3/2: (1 + c r) exp(-c r), which is
// 1 at r = 0 (taken exactly there, where the square root has no derivative).
template <class T>
T kernel_r2(int kernel, const T& r2, const T& ell) {
  if (kernel == KERNEL_RBF) return exp(-r2 / (T(2.0) * ell * ell));
  if (!(val(r2) > 0)) return T(1.0);
  const T t = matern_rate(ell) * sqrt(r2);
  return (T(1.0) + t) * exp(-t);
}

// ---------------------------------------------------------------------------
// fit: A = K + Sigma (eq. log_gp_posterior_mean with K_ij = k(x_i, x_j), Sigma_ii =
// sigma_i^2), k from Table I; A = L L^T (textbook Cholesky); a = A^{-1} 1 (all
// labels equal exp(-lambda * 0) = 1).
// ---------------------------------------------------------------------------
struct Inputs {
  const double* pts;        // [N,3] surface samples
  const double* svar;       // [N] per-sample sigma_i^2 or null (uniform)
  int n_cells;
  const int* offsets;       // [n_cells+1]
  const int* samples;       // [nnz]
  const double* centres;    // [n_cells,3]
  const long* lofs;         // [n_cells] offset of each cell's m x m factor
  int kernel;               // KERNEL_RBF or KERNEL_MATERN32
};

template <class T>
T sample_var(const Inputs& in, int s, const T& noise) {
  return in.svar ? T(in.svar[s]) : noise;
}

// Returns false when a pivot is not positive (cell not SPD).
// A = K + Sigma of cell c, row-major m x m.
template <class T>
std::vector<T> assemble_cell(const Inputs& in, int c, const T& ell, const T& noise) {
  const int b = in.offsets[c], m = in.offsets[c + 1] - b;
  std::vector<T> A((size_t)m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      const double* xi = in.pts + 3 * (long)in.samples[b + i];
      const double* xj = in.pts + 3 * (long)in.samples[b + j];
      double dx = xi[0] - xj[0], dy = xi[1] - xj[1], dz = xi[2] - xj[2];
      double r2 = dx * dx + dy * dy + dz * dz;
      A[(size_t)i * m + j] = i == j ? T(1.0) : kernel_r2(in.kernel, T(r2), ell);
      if (i == j) A[(size_t)i * m + j] = A[(size_t)i * m + j] + sample_var(in, in.samples[b + i], noise);
    }
  return A;
}

template <class T>
bool fit_cell(const Inputs& in, int c, const T& ell, const T& noise, T* a, T* L) {
  const int m = in.offsets[c + 1] - in.offsets[c];
  std::vector<T> A = assemble_cell(in, c, ell, noise);
  for (int i = 0; i < m * m; ++i) L[i] = T(0.0);
  for (int j = 0; j < m; ++j) {
    T s = A[(size_t)j * m + j];
    for (int k = 0; k < j; ++k) s = s - L[(size_t)j * m + k] * L[(size_t)j * m + k];
    if (!(val(s) > 0)) return false;
    L[(size_t)j * m + j] = sqrt(s);
    for (int i = j + 1; i < m; ++i) {
      T t = A[(size_t)i * m + j];
      for (int k = 0; k < j; ++k) t = t - L[(size_t)i * m + k] * L[(size_t)j * m + k];
      L[(size_t)i * m + j] = t / L[(size_t)j * m + j];
    }
  }
  std::vector<T> y(m);
  for (int i = 0; i < m; ++i) {            // L y = 1
    T t = T(1.0);
    for (int k = 0; k < i; ++k) t = t - L[(size_t)i * m + k] * y[k];
    y[i] = t / L[(size_t)i * m + i];
  }
  for (int i = m - 1; i >= 0; --i) {       // L^T a = y
    T t = y[i];
    for (int k = i + 1; k < m; ++k) t = t - L[(size_t)k * m + i] * a[k];
    a[i] = t / L[(size_t)i * m + i];
  }
  return true;
}

// ---------------------------------------------------------------------------
// query
// ---------------------------------------------------------------------------
struct QueryOpts {
  double ell_v, alpha_v;
  int k_fuse;
  double tie_rel;       // relative width of the tie band at the K-th distance (R6)
  int d_mode;           // 0: d = nearest sample (default); 1: d = first sample; 2: d = 0
  bool alpha_tied;      // alpha = 1/(2 l^2) follows l
};

// The K nearest occupied cell centres by exact (double) distance, ties by lower id
// (Sec. IV-B.1, "K nearest GPs").  Reading R6: when the K-th place is tied, i.e.
// more cells than the free places lie within tie_rel of the K-th distance, any
// choice of those tied cells is an acceptable candidate set.  `list` then holds the
// strictly nearer cells followed by the whole tie group (n_def + n_tie cells, of
// which n_pick tied cells join the set); otherwise it is the K nearest.  `kset` is
// always the K nearest with ties broken by id.
struct CandSet {
  std::vector<int> kset, list;
  int n_def = 0, n_tie = 0, n_pick = 0;
};

CandSet candidates(const Inputs& in, const double* q, const QueryOpts& o) {
  CandSet cs;
  std::vector<std::pair<double, int>> d(in.n_cells);
  for (int c = 0; c < in.n_cells; ++c) {
    const double* ce = in.centres + 3 * (long)c;
    double dx = q[0] - ce[0], dy = q[1] - ce[1], dz = q[2] - ce[2];
    d[c] = {dx * dx + dy * dy + dz * dz, c};
  }
  const int k = std::min(o.k_fuse, in.n_cells);
  if (k == 0) return cs;
  std::nth_element(d.begin(), d.begin() + (k - 1), d.end());
  const double dk2 = d[k - 1].first;
  const double hi2 = dk2 * (1.0 + o.tie_rel) * (1.0 + o.tie_rel);
  const double lo2 = dk2 * (1.0 - o.tie_rel) * (1.0 - o.tie_rel);
  std::vector<std::pair<double, int>> near;
  for (const auto& e : d)
    if (e.first <= hi2) near.push_back(e);
  std::sort(near.begin(), near.end());
  for (int i = 0; i < k; ++i) cs.kset.push_back(near[i].second);
  int n_def = 0, n_tie = 0;
  for (const auto& e : near) (e.first < lo2 ? n_def : n_tie) += 1;
  if (n_tie > k - n_def) {
    for (const auto& e : near) cs.list.push_back(e.second);
    cs.n_def = n_def;
    cs.n_tie = n_tie;
    cs.n_pick = k - n_def;
  } else {
    cs.list = cs.kset;
    cs.n_def = k;
  }
  return cs;
}

// Per-candidate UDF (eq. log_gp_posterior_mean mean with App. D scaling, Table I transform).
template <class T>
T cell_udf(const Inputs& in, int c, const T* q, const T* a, const T& ell, const QueryOpts& o,
           bool* clamped) {
  const int b = in.offsets[c], m = in.offsets[c + 1] - b;
  std::vector<T> z2(m);
  for (int i = 0; i < m; ++i) {
    const double* x = in.pts + 3 * (long)in.samples[b + i];
    T dx = q[0] - T(x[0]), dy = q[1] - T(x[1]), dz = q[2] - T(x[2]);
    z2[i] = dx * dx + dy * dy + dz * dz;
  }
  T d2 = T(0.0);
  if (o.d_mode == 0) {
    d2 = z2[0];
    for (int i = 1; i < m; ++i) if (val(z2[i]) < val(d2)) d2 = z2[i];
  } else if (o.d_mode == 1) {
    d2 = z2[0];
  }
  T f = T(0.0);
  if (in.kernel == KERNEL_MATERN32) {
    // f' = gamma f with gamma = exp(c d): sum a_i (1 + c z_i) exp(-c (z_i - d));
    // u = d - log(f') / c (App. D, Table I)
    const T c = matern_rate(ell);
    const T d = sqrt(d2);
    for (int i = 0; i < m; ++i) {
      const T z = sqrt(z2[i]);
      f = f + a[b + i] * (T(1.0) + c * z) * exp(-c * (z - d));
    }
    if (!(val(f) > 0)) return T(std::numeric_limits<double>::infinity());
    T u = d - log(f) / c;
    if (val(u) < 0) { if (clamped) *clamped = true; return T(0.0); }
    if (clamped) *clamped = false;
    return u;
  }
  for (int i = 0; i < m; ++i) f = f + a[b + i] * exp(-(z2[i] - d2) / (T(2.0) * ell * ell));
  if (!(val(f) > 0)) return T(std::numeric_limits<double>::infinity());
  T u2 = d2 - T(2.0) * ell * ell * log(f);
  if (val(u2) < 0) { if (clamped) *clamped = true; return T(0.0); }
  if (clamped) *clamped = false;
  return sqrt(u2);
}

template <class T>
struct CellOut {
  T grad[3];
  T var, var_f;
  T grad_var[3];         // V[grad_k u] of App. C
  double ratio;          // cancellation ratio sum|a_i| e_i |x*-x_i| / |w|
  double fratio;         // cancellation ratio of the scaled mean: sum|a_i e_i| / |sum a_i e_i|
  bool grad_zero;
};

// Gradient, GP variance and softmin SDF variance of one cell at q.
template <class T>
CellOut<T> cell_outputs(const Inputs& in, int c, const T* q, const T* a, const T* L,
                        const T& ell, const T& noise, const T& alpha, const QueryOpts& o) {
  const int b = in.offsets[c], m = in.offsets[c + 1] - b;
  std::vector<T> z2(m), diff(3 * (size_t)m);
  for (int i = 0; i < m; ++i) {
    const double* x = in.pts + 3 * (long)in.samples[b + i];
    for (int d = 0; d < 3; ++d) diff[3 * i + d] = q[d] - T(x[d]);
    z2[i] = diff[3 * i] * diff[3 * i] + diff[3 * i + 1] * diff[3 * i + 1] + diff[3 * i + 2] * diff[3 * i + 2];
  }
  T d2 = z2[0];
  for (int i = 1; i < m; ++i) if (val(z2[i]) < val(d2)) d2 = z2[i];
  if (o.d_mode == 1) d2 = z2[0];
  if (o.d_mode == 2) d2 = T(0.0);
  CellOut<T> r;
  // gradient.  RBF: grad f = -(1/l^2) sum a_i k_i (x* - x_i); Matern 3/2: dk/dr =
  // -c^2 r exp(-c r), so grad f = -c^2 sum a_i exp(-c z_i) (x* - x_i).  Either way the
  // UDF gradient is -grad f / |grad f| = w / |w| with w = sum a_i e_i (x* - x_i),
  // e_i = k_i (RBF) or exp(-c z_i) (Matern), both scaled by gamma.
  const bool matern = in.kernel == KERNEL_MATERN32;
  const T cm = matern_rate(ell);
  const T dref = matern ? sqrt(d2) : T(0.0);
  T w[3] = {T(0.0), T(0.0), T(0.0)};
  double absum = 0, fabs_sum = 0, fsum = 0;
  for (int i = 0; i < m; ++i) {
    T e = matern ? exp(-cm * (sqrt(z2[i]) - dref)) : exp(-(z2[i] - d2) / (T(2.0) * ell * ell));
    for (int d = 0; d < 3; ++d) w[d] = w[d] + a[b + i] * e * diff[3 * i + d];
    absum += std::fabs(val(a[b + i]) * val(e)) * std::sqrt(val(z2[i]));
    fabs_sum += std::fabs(val(a[b + i]) * val(e));
    fsum += val(a[b + i]) * val(e);
  }
  r.fratio = fsum != 0 ? fabs_sum / std::fabs(fsum) : std::numeric_limits<double>::infinity();
  T wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  r.grad_zero = !(val(wn) > 0);
  for (int d = 0; d < 3; ++d) r.grad[d] = r.grad_zero ? T(0.0) : w[d] / wn;
  r.ratio = r.grad_zero ? std::numeric_limits<double>::infinity() : absum / val(wn);
  // GP variance: k(x*, x*) - k*^T (K + Sigma)^{-1} k* = 1 - |L^{-1} k*|^2 (unscaled k*).
  std::vector<T> v(m);
  T vv = T(0.0);
  for (int i = 0; i < m; ++i) {
    T t = kernel_r2(in.kernel, z2[i], ell);
    for (int k = 0; k < i; ++k) t = t - L[in.lofs[c] + (long)i * m + k] * v[k];
    v[i] = t / L[in.lofs[c] + (long)i * m + i];
    vv = vv + v[i] * v[i];
  }
  r.var_f = T(1.0) - vv;
  if (val(r.var_f) < 0) r.var_f = T(0.0);
  // softmin SDF variance: s = softmax(-alpha z), h = s^T z,
  // grad_{x_i} h = -s_i (alpha h - alpha z_i + 1)(x* - x_i)/z_i, |.|^2 = c_i^2.
  std::vector<T> z(m), s(m);
  T zmin = T(0.0);
  for (int i = 0; i < m; ++i) {
    z[i] = sqrt(z2[i]);
    if (i == 0 || val(z[i]) < val(zmin)) zmin = z[i];
  }
  T ssum = T(0.0);
  for (int i = 0; i < m; ++i) { s[i] = exp(-alpha * (z[i] - zmin)); ssum = ssum + s[i]; }
  T hval = T(0.0);
  for (int i = 0; i < m; ++i) { s[i] = s[i] / ssum; hval = hval + s[i] * z[i]; }
  T var = T(0.0);
  for (int i = 0; i < m; ++i) {
    T ci = s[i] * (alpha * hval - alpha * z[i] + T(1.0));
    var = var + ci * ci * sample_var(in, in.samples[b + i], noise);
  }
  r.var = var;
  // SDF gradient variance (App. C, the variance of the softmin gradient): with
  // v_i = (x* - x_i)/z_i, l_i = s_i (alpha h - alpha z_i + 1) and g = sum_i l_i v_i,
  // the derivative of g with respect to sample x_i (rows: components of g) is
  //   J_i = alpha w_i v_i^T + (l_i / z_i)(v_i v_i^T - I),  w_i = l_i (v_i - V s) + s_i (v_i - g)
  // (App. C prints its transpose, the gradient layout), and
  //   V[grad_k u] = sum_i sigma_i^2 |row k of J_i|^2.
  // A sample at the query itself (z_i = 0) has no direction and contributes nothing.
  std::vector<T> vdir(3 * (size_t)m, T(0.0));
  T Vs[3] = {T(0.0), T(0.0), T(0.0)}, gs[3] = {T(0.0), T(0.0), T(0.0)};
  std::vector<T> li(m);
  for (int i = 0; i < m; ++i) {
    li[i] = s[i] * (alpha * hval - alpha * z[i] + T(1.0));
    if (val(z[i]) > 0)
      for (int d = 0; d < 3; ++d) vdir[3 * i + d] = diff[3 * i + d] / z[i];
    for (int d = 0; d < 3; ++d) {
      Vs[d] = Vs[d] + s[i] * vdir[3 * i + d];
      gs[d] = gs[d] + li[i] * vdir[3 * i + d];
    }
  }
  for (int k = 0; k < 3; ++k) r.grad_var[k] = T(0.0);
  for (int i = 0; i < m; ++i) {
    if (!(val(z[i]) > 0)) continue;
    T wv[3];
    for (int d = 0; d < 3; ++d)
      wv[d] = li[i] * (vdir[3 * i + d] - Vs[d]) + s[i] * (vdir[3 * i + d] - gs[d]);
    const T sv2 = sample_var(in, in.samples[b + i], noise);
    for (int k = 0; k < 3; ++k) {
      T row2 = T(0.0);
      for (int j = 0; j < 3; ++j) {
        const T Jkj = alpha * wv[k] * vdir[3 * i + j] +
                      (li[i] / z[i]) * (vdir[3 * i + k] * vdir[3 * i + j] - T(k == j ? 1.0 : 0.0));
        row2 = row2 + Jkj * Jkj;
      }
      r.grad_var[k] = r.grad_var[k] + sv2 * row2;
    }
  }
  return r;
}

template <class T>
struct PointOut {
  T mean, grad[3], var, var_f, grad_var[3];
  int argmin;
  double u_best, u_second, ratio, fratio;
  int status;
  CandSet cs;                     // the candidate set and its R6 tie group
  std::vector<double> ucand;      // u of every cell of cs.list
  std::vector<CellOut<T>> cout;   // per-cell outputs of cs.list (when requested)
  int forced = -1;                // 1: the forced cell was used; 0: it was not in cs.list or invalid
};

enum { ST_NO_VALID = 1, ST_CLAMPED = 2, ST_GRAD_ZERO = 4 };

// Outputs at one query.  The fused u is the minimum over the K nearest cells (ties by
// id, also among equal u).  A forced cell (a near-tie of the candidate set or of the
// min-fusion resolved the other way, which the caller has checked against the
// tolerance) replaces the minimum when it is one of cs.list with a finite u.
template <class T>
PointOut<T> query_point(const Inputs& in, const T* q, int sign, const T* a, const T* L,
                        const T& ell, const T& noise, const T& alpha, const QueryOpts& o,
                        bool all_candidates = false, int forced = -1) {
  double qv[3] = {val(q[0]), val(q[1]), val(q[2])};
  PointOut<T> r;
  r.status = 0;
  r.cs = candidates(in, qv, o);
  std::vector<T> ul(r.cs.list.size());
  std::vector<bool> clamp(r.cs.list.size(), false);
  for (size_t i = 0; i < r.cs.list.size(); ++i) {
    bool cl = false;
    ul[i] = cell_udf(in, r.cs.list[i], q, a, ell, o, &cl);
    clamp[i] = cl;
    r.ucand.push_back(val(ul[i]));
  }
  if (all_candidates)
    for (int c : r.cs.list) {
      CellOut<T> co = cell_outputs(in, c, q, a, L, ell, noise, alpha, o);
      for (int d = 0; d < 3; ++d) co.grad[d] = T((double)sign) * co.grad[d];
      r.cout.push_back(co);
    }
  // the K nearest, ordered by (u, id)
  std::vector<std::pair<double, int>> us;   // (u, position in cs.list)
  for (size_t i = 0; i < r.cs.list.size(); ++i)
    if (std::find(r.cs.kset.begin(), r.cs.kset.end(), r.cs.list[i]) != r.cs.kset.end())
      us.push_back({r.ucand[i], (int)i});
  std::sort(us.begin(), us.end(), [&](const auto& x, const auto& y) {
    return std::make_pair(x.first, r.cs.list[x.second]) < std::make_pair(y.first, r.cs.list[y.second]);
  });
  const double inf = std::numeric_limits<double>::infinity();
  r.argmin = -1; r.u_best = inf; r.u_second = inf; r.ratio = inf; r.fratio = inf;
  if (us.size() > 1) r.u_second = us[1].first;
  int pick = us.empty() ? -1 : us[0].second;
  if (forced >= 0) {
    r.forced = 0;
    for (size_t i = 0; i < r.cs.list.size(); ++i)
      if (r.cs.list[i] == forced && r.ucand[i] < inf) { pick = (int)i; r.forced = 1; }
  }
  if (pick < 0 || !(r.ucand[pick] < inf)) {
    r.status = ST_NO_VALID;
    r.mean = T(inf);
    for (int d = 0; d < 3; ++d) r.grad[d] = T(0.0);
    r.var = T(inf); r.var_f = T(1.0);
    for (int d = 0; d < 3; ++d) r.grad_var[d] = T(inf);
    return r;
  }
  r.argmin = r.cs.list[pick];
  r.u_best = r.ucand[pick];
  if (clamp[pick]) r.status |= ST_CLAMPED;
  // d = s * u; grad d = s * grad u; V[d] = V[u] (deterministic sign).
  r.mean = T((double)sign) * ul[pick];
  CellOut<T> co = cell_outputs(in, r.argmin, q, a, L, ell, noise, alpha, o);
  for (int d = 0; d < 3; ++d) r.grad[d] = T((double)sign) * co.grad[d];
  r.var = co.var; r.var_f = co.var_f; r.ratio = co.ratio; r.fratio = co.fratio;
  for (int d = 0; d < 3; ++d) r.grad_var[d] = co.grad_var[d];
  if (co.grad_zero) r.status |= ST_GRAD_ZERO;
  return r;
}

// Eigenvalues of a symmetric m x m matrix (row-major) by the cyclic Jacobi method:
// sweeps of plane rotations, each zeroing one off-diagonal pair, until the
// off-diagonal mass is negligible against the whole (Golub and Van Loan, Matrix
// Computations, Sec. 8.5).  Accurate to about machine precision times the norm.
std::vector<double> sym_eigenvalues(std::vector<double> A, int m) {
  auto at = [&](int i, int j) -> double& { return A[(size_t)i * m + j]; };
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0, all = 0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        all += at(i, j) * at(i, j);
        if (i != j) off += at(i, j) * at(i, j);
      }
    if (off <= 1e-32 * all) break;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = at(p, q);
        if (apq == 0) continue;
        // the rotation angle that zeroes (p, q): tan of it is the smaller root of
        // t^2 + 2 tau t - 1 = 0 with tau = (a_qq - a_pp) / (2 a_pq)
        const double tau = (at(q, q) - at(p, p)) / (2 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1 + tau * tau));
        const double cs = 1 / std::sqrt(1 + t * t), sn = t * cs;
        for (int k = 0; k < m; ++k) {        // A <- A J
          const double kp = at(k, p), kq = at(k, q);
          at(k, p) = cs * kp - sn * kq;
          at(k, q) = sn * kp + cs * kq;
        }
        for (int k = 0; k < m; ++k) {        // A <- J^T A
          const double pk = at(p, k), qk = at(q, k);
          at(p, k) = cs * pk - sn * qk;
          at(q, k) = sn * pk + cs * qk;
        }
      }
  }
  std::vector<double> ev(m);
  for (int i = 0; i < m; ++i) ev[i] = at(i, i);
  return ev;
}

Inputs make_inputs(const double* pts, const double* svar, int n_cells, const int* offsets,
                   const int* samples, const double* centres, std::vector<long>& lofs,
                   int kernel) {
  lofs.assign(n_cells + 1, 0);
  for (int c = 0; c < n_cells; ++c) {
    long m = offsets[c + 1] - offsets[c];
    lofs[c + 1] = lofs[c] + m * m;
  }
  return Inputs{pts, svar, n_cells, offsets, samples, centres, lofs.data(), kernel};
}

template <class T>
int fit_all(const Inputs& in, const T& ell, const T& noise, std::vector<T>& a, std::vector<T>& L,
            int* ok) {
  a.assign(in.offsets[in.n_cells], T(0.0));
  L.assign(in.lofs[in.n_cells], T(0.0));
  int nfail = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : nfail)
  for (int c = 0; c < in.n_cells; ++c) {
    bool good = fit_cell(in, c, ell, noise, a.data() + in.offsets[c], L.data() + in.lofs[c]);
    if (ok) ok[c] = good ? 1 : 0;
    if (!good) {
      // a failed cell is excluded: all-zero weights give f' = 0 -> u = +inf.
      for (int i = in.offsets[c]; i < in.offsets[c + 1]; ++i) a[i] = T(0.0);
      for (long i = in.lofs[c]; i < in.lofs[c + 1]; ++i) L[i] = T(1.0);
      ++nfail;
    }
  }
  return nfail;
}

double softplus(double t) { return std::max(t, 0.0) + std::log1p(std::exp(-std::fabs(t))); }
template <int N> Dual<N> softplus(const Dual<N>& t) {
  Dual<N> m = t.v > 0 ? t : Dual<N>(0.0);
  return m + log1p(exp(-fabs(t)));
}

}  // namespace

extern "C" {

// Softmin distance h = s^T z (s = softmax(-alpha z), z_i = |q - x_i|) of a sample set and
// its gradient g = grad_q h = sum_i l_i v_i (Sec. IV-B.3, App. C), for tests of the
// gradient variance by finite differences.
void oracle_softmin(const double* q, const double* x, int m, double alpha, double* h, double* g) {
  std::vector<double> z(m), sm(m);
  double zmin = 0, ssum = 0, hv = 0;
  for (int i = 0; i < m; ++i) {
    double d2 = 0;
    for (int d = 0; d < 3; ++d) d2 += (q[d] - x[3 * i + d]) * (q[d] - x[3 * i + d]);
    z[i] = std::sqrt(d2);
    if (i == 0 || z[i] < zmin) zmin = z[i];
  }
  for (int i = 0; i < m; ++i) { sm[i] = std::exp(-alpha * (z[i] - zmin)); ssum += sm[i]; }
  for (int i = 0; i < m; ++i) { sm[i] /= ssum; hv += sm[i] * z[i]; }
  *h = hv;
  for (int d = 0; d < 3; ++d) g[d] = 0;
  for (int i = 0; i < m; ++i) {
    const double li = sm[i] * (alpha * hv - alpha * z[i] + 1.0);
    if (z[i] > 0)
      for (int d = 0; d < 3; ++d) g[d] += li * (q[d] - x[3 * i + d]) / z[i];
  }
}

// Log-odds of local Bayesian Hilbert maps and the SDF sign (Sec. IV-A, eq.
// sign_prediction; App. B features): l(x) = mu^T phi(x), phi = [k(x, h_1) .. k(x, h_M), 1]
// with k(x, h) = exp(-gamma |x - h|^2) over the hinge points of the map of the box
// holding x (box lattice from `origin`, edge `box`, `dims` boxes per axis; hinges^3
// points at the box's lattice points, spacing box / (hinges - 1); weights per map
// hinges^3 + 1 with the bias last).  sign = +1 where l < tau, else -1; +1 and
// have = 0 where the box has no map.
void oracle_bhm(const double* origin, double box, const int* dims, int hinges, double gamma,
                const int* box_bhm, const double* weights, const double* q, long nq, double tau,
                double* logodds, int* have, int* sign) {
  const double sp = box / (double)(hinges - 1);
  const long m = (long)hinges * hinges * hinges;
  for (long p = 0; p < nq; ++p) {
    const double* x = q + 3 * p;
    long key[3];
    bool in = true;
    for (int d = 0; d < 3; ++d) {
      key[d] = (long)std::floor((x[d] - origin[d]) / box);
      in = in && key[d] >= 0 && key[d] < dims[d];
    }
    const int id = in ? box_bhm[(key[0] * dims[1] + key[1]) * dims[2] + key[2]] : -1;
    have[p] = id >= 0;
    double l = 0;
    if (id >= 0) {
      const double* w = weights + (long)id * (m + 1);
      for (int i = 0; i < hinges; ++i)
        for (int j = 0; j < hinges; ++j)
          for (int k = 0; k < hinges; ++k) {
            const double h[3] = {origin[0] + (double)key[0] * box + i * sp,
                                 origin[1] + (double)key[1] * box + j * sp,
                                 origin[2] + (double)key[2] * box + k * sp};
            double d2 = 0;
            for (int d = 0; d < 3; ++d) d2 += (x[d] - h[d]) * (x[d] - h[d]);
            l += w[((long)i * hinges + j) * hinges + k] * std::exp(-gamma * d2);
          }
      l += w[m];
    }
    logodds[p] = l;
    sign[p] = (id < 0 || l < tau) ? 1 : -1;
  }
}

// Worker threads the parallel loops below use.
int oracle_threads() { return omp_get_max_threads(); }

// Fit every cell in FP64.  a: [nnz]; L: concatenated row-major m_c x m_c factors.
// kernel: KERNEL_RBF (0) or KERNEL_MATERN32 (1), here and below.
int oracle_fit(const double* pts, const double* svar, int n_cells, const int* offsets,
               const int* samples, double ell, double noise, double* a_out, double* L_out,
               int* ok, int kernel) {
  std::vector<long> lofs;
  Inputs in = make_inputs(pts, svar, n_cells, offsets, samples, nullptr, lofs, kernel);
  std::vector<double> a, L;
  int nfail = fit_all<double>(in, ell, noise, a, L, ok);
  std::copy(a.begin(), a.end(), a_out);
  if (L_out) std::copy(L.begin(), L.end(), L_out);
  return nfail;
}

// Query every point.  Outputs per query: mean, grad[3], var, var_f, argmin, status,
// the best and second-best u among the K nearest, the cancellation ratios of the
// argmin cell's direction and mean, and the candidate list (the K nearest, or with a
// tie at the K-th place the nearer cells and the whole tie group; width cw, -1
// padded) with each cell's u; tie[3] = (n_def, n_tie, n_pick) of the list (n_tie =
// 0: no tie); and (when cgrad is given) every listed cell's gradient, variances and
// ratio, for near-tie acceptance.  Returns the number of queries whose list did not
// fit in cw.
long oracle_query(const double* pts, const double* svar, int n_cells, const int* offsets,
                  const int* samples, const double* centres, const double* a_in,
                  const double* L_in, double ell, double noise, double alpha, int k_fuse,
                  double tie_rel, int d_mode, const double* q, long nq, const int8_t* sign,
                  double* mean, double* grad, double* var, double* var_f, int* argmin,
                  int* status, double* u_best, double* u_second, double* ratio, double* fratio,
                  int cw, int* cand, double* ucand, int* tie, double* cgrad, double* cvar,
                  double* cvar_f, double* cratio, double* grad_var, double* cgrad_var, int kernel) {
  std::vector<long> lofs;
  Inputs in = make_inputs(pts, svar, n_cells, offsets, samples, centres, lofs, kernel);
  QueryOpts o{ell, alpha, k_fuse, tie_rel, d_mode, false};
  const double inf = std::numeric_limits<double>::infinity();
  long overflow = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : overflow)
  for (long p = 0; p < nq; ++p) {
    PointOut<double> r = query_point<double>(in, q + 3 * p, sign ? sign[p] : 1, a_in, L_in,
                                             ell, noise, alpha, o, cgrad != nullptr);
    mean[p] = r.mean; var[p] = r.var; var_f[p] = r.var_f;
    for (int d = 0; d < 3; ++d) grad[3 * p + d] = r.grad[d];
    if (grad_var)
      for (int d = 0; d < 3; ++d) grad_var[3 * p + d] = r.grad_var[d];
    argmin[p] = r.argmin; status[p] = r.status;
    if (u_best) u_best[p] = r.u_best;
    if (u_second) u_second[p] = r.u_second;
    if (ratio) ratio[p] = r.ratio;
    if (fratio) fratio[p] = r.fratio;
    if (tie) {
      tie[3 * p] = r.cs.n_def; tie[3 * p + 1] = r.cs.n_tie; tie[3 * p + 2] = r.cs.n_pick;
    }
    if ((int)r.cs.list.size() > cw) ++overflow;
    for (int i = 0; i < cw; ++i) {
      bool have = i < (int)r.cs.list.size();
      long j = (long)cw * p + i;
      if (cand) cand[j] = have ? r.cs.list[i] : -1;
      if (ucand) ucand[j] = have ? r.ucand[i] : inf;
      if (cgrad) {
        for (int d = 0; d < 3; ++d) cgrad[3 * j + d] = have ? r.cout[i].grad[d] : 0.0;
        cvar[j] = have ? r.cout[i].var : inf;
        cvar_f[j] = have ? r.cout[i].var_f : 1.0;
        cratio[j] = have ? r.cout[i].ratio : inf;
        if (cgrad_var)
          for (int d = 0; d < 3; ++d) cgrad_var[3 * j + d] = have ? r.cout[i].grad_var[d] : inf;
      }
    }
  }
  return overflow;
}

// Exact 2-norm condition number of every cell's A = K + Sigma (the matrix the fit
// factors): the ratio of its extreme eigenvalues from cyclic Jacobi rotations; +inf
// where the smallest eigenvalue is not positive.
// ids [n_ids] selects the cells (null: every cell, n_ids ignored); outputs follow ids.
void oracle_cond2(const double* pts, const double* svar, int n_cells, const int* offsets,
                  const int* samples, double ell, double noise, int kernel, const int* ids,
                  long n_ids, double* cond, double* eig_min, double* eig_max) {
  std::vector<long> lofs;
  Inputs in = make_inputs(pts, svar, n_cells, offsets, samples, nullptr, lofs, kernel);
  const long n = ids ? n_ids : n_cells;
#pragma omp parallel for schedule(dynamic, 1)
  for (long j = 0; j < n; ++j) {
    const int c = ids ? ids[j] : (int)j;
    const int m = offsets[c + 1] - offsets[c];
    std::vector<double> ev = sym_eigenvalues(assemble_cell<double>(in, c, ell, noise), m);
    const double lo = *std::min_element(ev.begin(), ev.end());
    const double hi = *std::max_element(ev.begin(), ev.end());
    cond[j] = lo > 0 ? hi / lo : std::numeric_limits<double>::infinity();
    if (eig_min) eig_min[j] = lo;
    if (eig_max) eig_max[j] = hi;
  }
}

// Vector-Jacobian product by forward-mode dual numbers.
//   mode 0: L = sum_q d_mean*mean + d_grad.grad + d_var*var + d_var_f*var_f
//   mode 1: L = sum_q softplus(margin - mean + weight*sqrt(var))   (cotangent args unused)
// d_points [nq,3] = dL/dq; d_hyper[2] = dL/d(l, sigma^2) through the fit as well
// (the whole fit is redone in dual arithmetic); alpha = 1/(2 l^2) follows l
// unless alpha_fixed > 0.  force_argmin [nq] (or null; -1 = none) differentiates at
// that cell where it is one of the query's listed candidates (see query_point);
// forced_used [nq] (or null) receives 1 where it was used, 0 where it was not, -1
// where none was given.  Returns L.
double oracle_vjp(const double* pts, int n_cells, const int* offsets, const int* samples,
                  const double* centres, double ell, double noise, double alpha_fixed,
                  int k_fuse, double tie_rel, const double* q, long nq, const int8_t* sign,
                  int mode, double margin, double weight, const double* d_mean,
                  const double* d_grad, const double* d_var, const double* d_var_f,
                  double* d_points, double* d_hyper, double* d_hyper_pp,
                  const int* force_argmin, int* forced_used, int kernel) {
  std::vector<long> lofs;
  Inputs in = make_inputs(pts, nullptr, n_cells, offsets, samples, centres, lofs, kernel);
  QueryOpts o{ell, 0, k_fuse, tie_rel, 0, alpha_fixed <= 0};
  auto loss_of = [&](long p, auto mean, auto* g, auto var, auto var_f) {
    using T = decltype(mean);
    if (mode == 1) return softplus(T(margin) - mean + T(weight) * sqrt(var));
    T l = T(d_mean ? d_mean[p] : 0.0) * mean + T(d_var ? d_var[p] : 0.0) * var +
          T(d_var_f ? d_var_f[p] : 0.0) * var_f;
    if (d_grad) for (int d = 0; d < 3; ++d) l = l + T(d_grad[3 * p + d]) * g[d];
    return l;
  };
  // (1) hyperparameters: fit and queries in Dual<2>.
  using D2 = Dual<2>;
  D2 ell2(ell); ell2.d[0] = 1.0;
  D2 noise2(noise); noise2.d[1] = 1.0;
  D2 alpha2 = alpha_fixed > 0 ? D2(alpha_fixed) : D2(1.0) / (D2(2.0) * ell2 * ell2);
  std::vector<D2> a2, L2;
  fit_all<D2>(in, ell2, noise2, a2, L2, nullptr);
  double total = 0, dh0 = 0, dh1 = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total, dh0, dh1)
  for (long p = 0; p < nq; ++p) {
    D2 qd[3] = {D2(q[3 * p]), D2(q[3 * p + 1]), D2(q[3 * p + 2])};
    PointOut<D2> r = query_point<D2>(in, qd, sign ? sign[p] : 1, a2.data(), L2.data(), ell2,
                                     noise2, alpha2, o, false, force_argmin ? force_argmin[p] : -1);
    if (r.status & ST_NO_VALID) {
      if (d_hyper_pp) d_hyper_pp[2 * p] = d_hyper_pp[2 * p + 1] = 0.0;
      continue;
    }
    D2 l = loss_of(p, r.mean, r.grad, r.var, r.var_f);
    total += l.v; dh0 += l.d[0]; dh1 += l.d[1];
    if (d_hyper_pp) {
      d_hyper_pp[2 * p] = l.d[0];
      d_hyper_pp[2 * p + 1] = l.d[1];
    }
  }
  d_hyper[0] = dh0; d_hyper[1] = dh1;
  // (2) query points: fit fixed in double, queries in Dual<3>.
  std::vector<double> a, L;
  fit_all<double>(in, ell, noise, a, L, nullptr);
  using D3 = Dual<3>;
  std::vector<D3> a3(a.begin(), a.end()), L3(L.begin(), L.end());
  D3 ell3(ell), noise3(noise);
  D3 alpha3 = alpha_fixed > 0 ? D3(alpha_fixed) : D3(1.0) / (D3(2.0) * ell3 * ell3);
#pragma omp parallel for schedule(dynamic, 64)
  for (long p = 0; p < nq; ++p) {
    D3 qd[3];
    for (int d = 0; d < 3; ++d) { qd[d] = D3(q[3 * p + d]); qd[d].d[d] = 1.0; }
    PointOut<D3> r = query_point<D3>(in, qd, sign ? sign[p] : 1, a3.data(), L3.data(), ell3,
                                     noise3, alpha3, o, false, force_argmin ? force_argmin[p] : -1);
    if (forced_used) forced_used[p] = r.forced;
    if (r.status & ST_NO_VALID) {
      for (int d = 0; d < 3; ++d) d_points[3 * p + d] = 0;
      continue;
    }
    D3 l = loss_of(p, r.mean, r.grad, r.var, r.var_f);
    for (int d = 0; d < 3; ++d) d_points[3 * p + d] = l.d[d];
  }
  return total;
}

}  // extern "C"
