// Host cell builder: the per-octant GP training buffers of Sec. IV-B.1.
//
// Every octant that holds surface samples trains its own GP on the samples inside
// a collection box larger than the octant, so neighbouring GPs share the samples
// near their common boundary.  Rule (see ksdf.h): key = floor((x - origin)/h);
// occupied keys own a cell; a cell's training set is the up-to-m_c samples of its
// box grown by `margin` (inclusive) nearest the centre, nearest first, ties by lower
// sample index; cells under m_min are dropped; ids in lexicographic key order.
//
// The selection is an integer decision taken from floating-point distances, so the
// expressions below are evaluated in double with contraction disabled: the same
// inputs always give the same cells.
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ksdf.h"

namespace ksdf {
void set_error(const std::string& msg);
}

struct ksdf_cellset {
  std::vector<int> offsets, samples, keys;
};

namespace {

struct K3 {
  long i, j, k;
  bool operator<(const K3& o) const { return std::tie(i, j, k) < std::tie(o.i, o.j, o.k); }
  bool operator==(const K3& o) const { return i == o.i && j == o.j && k == o.k; }
};

template <class T>
double coord(const void* p, long s, int d) {
  return (double)static_cast<const T*>(p)[3 * s + d];
}

}  // namespace

extern "C" int ksdf_build_cells(const void* pts, int dtype, long n, const double origin[3],
                                double h, double margin, int m_max, int m_min,
                                const uint8_t* cap_grid, const int key_lo[3],
                                const int key_dims[3], ksdf_cellset** out) {
  if (!out || (n > 0 && !pts) || !origin || !(h > 0) || !(margin >= 0) || m_max < 1 ||
      m_max > KSDF_MAX_M || m_min < 1 || (dtype != KSDF_DTYPE_F32 && dtype != KSDF_DTYPE_F64) ||
      (cap_grid && (!key_lo || !key_dims))) {
    ksdf::set_error("ksdf_build_cells: invalid argument");
    return KSDF_ERR_INVALID_ARGUMENT;
  }
  *out = nullptr;
  auto X = [&](long s, int d) {
    return dtype == KSDF_DTYPE_F32 ? coord<float>(pts, s, d) : coord<double>(pts, s, d);
  };
  for (long s = 0; s < n; ++s)
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(X(s, d))) {
        ksdf::set_error("ksdf_build_cells: non-finite surface point");
        return KSDF_ERR_INVALID_INPUT;
      }
  // bin samples by key: sort (key, index)
  std::vector<std::pair<K3, long>> keyed(n);
  for (long s = 0; s < n; ++s)
    keyed[s] = {K3{(long)std::floor((X(s, 0) - origin[0]) / h),
                   (long)std::floor((X(s, 1) - origin[1]) / h),
                   (long)std::floor((X(s, 2) - origin[2]) / h)},
                s};
  std::sort(keyed.begin(), keyed.end(), [](const auto& a, const auto& b) {
    return a.first < b.first || (a.first == b.first && a.second < b.second);
  });
  std::vector<K3> bin_key;
  std::vector<long> bin_start;
  for (long t = 0; t < n; ++t)
    if (t == 0 || !(keyed[t].first == keyed[t - 1].first)) {
      bin_key.push_back(keyed[t].first);
      bin_start.push_back(t);
    }
  bin_start.push_back(n);
  const long nb = (long)bin_key.size();
  auto find_bin = [&](const K3& k) -> long {
    auto it = std::lower_bound(bin_key.begin(), bin_key.end(), k);
    return (it != bin_key.end() && *it == k) ? (long)(it - bin_key.begin()) : -1;
  };
  const long reach = (long)std::ceil(margin / h) + 1;

  std::vector<std::vector<int>> sel(nb);
  auto work = [&](long b0, long b1) {
    std::vector<std::pair<double, long>> cand;
    for (long b = b0; b < b1; ++b) {
      const K3 c = bin_key[b];
      const long kc[3] = {c.i, c.j, c.k};
      double lo[3], hi[3], ctr[3];
      for (int d = 0; d < 3; ++d) {
        lo[d] = origin[d] + (double)kc[d] * h - margin;
        hi[d] = origin[d] + (double)(kc[d] + 1) * h + margin;
        ctr[d] = origin[d] + ((double)kc[d] + 0.5) * h;
      }
      cand.clear();
      for (long di = -reach; di <= reach; ++di)
        for (long dj = -reach; dj <= reach; ++dj)
          for (long dk = -reach; dk <= reach; ++dk) {
            long nbin = find_bin(K3{c.i + di, c.j + dj, c.k + dk});
            if (nbin < 0) continue;
            for (long t = bin_start[nbin]; t < bin_start[nbin + 1]; ++t) {
              const long s = keyed[t].second;
              const double x = X(s, 0), y = X(s, 1), z = X(s, 2);
              if (!(x >= lo[0] && x <= hi[0] && y >= lo[1] && y <= hi[1] && z >= lo[2] &&
                    z <= hi[2]))
                continue;
              const double dx = x - ctr[0], dy = y - ctr[1], dz = z - ctr[2];
              const double r2 = dx * dx + dy * dy + dz * dz;
              cand.push_back({r2, s});
            }
          }
      long m_c = m_max;
      if (cap_grid) {
        const long g0 = kc[0] - key_lo[0], g1 = kc[1] - key_lo[1], g2 = kc[2] - key_lo[2];
        if (g0 >= 0 && g0 < key_dims[0] && g1 >= 0 && g1 < key_dims[1] && g2 >= 0 &&
            g2 < key_dims[2])
          m_c = std::min<long>(m_max, cap_grid[(g0 * key_dims[1] + g1) * key_dims[2] + g2]);
      }
      const long take = std::min<long>(m_c, (long)cand.size());
      if (take < m_min) continue;
      std::partial_sort(cand.begin(), cand.begin() + take, cand.end());
      sel[b].resize(take);
      for (long t = 0; t < take; ++t) sel[b][t] = (int)cand[t].second;
    }
  };
  unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  if (nb < 256) nt = 1;
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) {
    long b0 = nb * t / nt, b1 = nb * (t + 1) / nt;
    if (nt == 1) work(b0, b1);
    else th.emplace_back(work, b0, b1);
  }
  for (auto& t : th) t.join();

  auto* cs = new ksdf_cellset;
  cs->offsets.push_back(0);
  for (long b = 0; b < nb; ++b) {
    if (sel[b].empty()) continue;
    cs->samples.insert(cs->samples.end(), sel[b].begin(), sel[b].end());
    cs->offsets.push_back((int)cs->samples.size());
    cs->keys.push_back((int)bin_key[b].i);
    cs->keys.push_back((int)bin_key[b].j);
    cs->keys.push_back((int)bin_key[b].k);
  }
  *out = cs;
  return KSDF_OK;
}

extern "C" int ksdf_cellset_info(const ksdf_cellset* cs, int* n_cells, long* nnz) {
  if (!cs || !n_cells || !nnz) return KSDF_ERR_INVALID_ARGUMENT;
  *n_cells = (int)cs->offsets.size() - 1;
  *nnz = (long)cs->samples.size();
  return KSDF_OK;
}

extern "C" int ksdf_cellset_copy(const ksdf_cellset* cs, int* offsets, int* samples, int* keys) {
  if (!cs || !offsets || (!samples && !cs->samples.empty()) || (!keys && !cs->keys.empty()))
    return KSDF_ERR_INVALID_ARGUMENT;
  std::memcpy(offsets, cs->offsets.data(), cs->offsets.size() * sizeof(int));
  if (!cs->samples.empty()) std::memcpy(samples, cs->samples.data(), cs->samples.size() * sizeof(int));
  if (!cs->keys.empty()) std::memcpy(keys, cs->keys.data(), cs->keys.size() * sizeof(int));
  return KSDF_OK;
}

extern "C" void ksdf_cellset_destroy(ksdf_cellset* cs) { delete cs; }
