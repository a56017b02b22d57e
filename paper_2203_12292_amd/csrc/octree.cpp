// Octree construction, closure and global coarsening (host side).
#include "octree.hpp"

#include <cmath>

#include "common.hpp"

namespace mfmg {

namespace {
inline void unkey(uint64_t key, int64_t& i, int64_t& j, int64_t& k) {
  const uint64_t m = (1ull << 21) - 1;
  i = static_cast<int64_t>((key >> 42) & m);
  j = static_cast<int64_t>((key >> 21) & m);
  k = static_cast<int64_t>(key & m);
}

void sort_unique(std::vector<uint64_t>& v) {
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
}

bool marked(const Octree& t, int l, int64_t i, int64_t j, int64_t k, int kind, const double* p) {
  const double h = (t.hi - t.lo) / (t.n0 * std::ldexp(1.0, l));
  const double cx = t.lo + (static_cast<double>(i) + 0.5) * h;
  const double cy = t.lo + (static_cast<double>(j) + 0.5) * h;
  const double cz = t.lo + (static_cast<double>(k) + 0.5) * h;
  switch (kind) {
    case MFMG_PRED_ALL:
      return true;
    case MFMG_PRED_BALL: {
      double d2 = (cx - p[0]) * (cx - p[0]) + (cy - p[1]) * (cy - p[1]) + (cz - p[2]) * (cz - p[2]);
      return d2 <= p[3] * p[3];
    }
    case MFMG_PRED_BOX_LE:
      return cx <= p[0] && cy <= p[1] && cz <= p[2];
    case MFMG_PRED_BAND: {
      double d2 = (cx - p[0]) * (cx - p[0]) + (cy - p[1]) * (cy - p[1]) + (cz - p[2]) * (cz - p[2]);
      return d2 >= p[3] * p[3] && d2 <= p[4] * p[4];
    }
    case MFMG_PRED_SPHERE_CUT: {
      double lo3[3] = {t.lo + static_cast<double>(i) * h, t.lo + static_cast<double>(j) * h,
                       t.lo + static_cast<double>(k) * h};
      double hi3[3] = {t.lo + (static_cast<double>(i) + 1.0) * h, t.lo + (static_cast<double>(j) + 1.0) * h,
                       t.lo + (static_cast<double>(k) + 1.0) * h};
      double dmin2 = 0, dmax2 = 0;
      for (int d = 0; d < 3; ++d) {
        double c = p[d];
        double nearest = std::min(std::max(c, lo3[d]), hi3[d]);
        dmin2 += (nearest - c) * (nearest - c);
        double far = (std::fabs(lo3[d] - c) > std::fabs(hi3[d] - c)) ? lo3[d] : hi3[d];
        dmax2 += (far - c) * (far - c);
      }
      bool m = dmin2 <= p[3] * p[3] && p[3] * p[3] <= dmax2;
      if (p[4] > 0) m = m || (dmin2 <= p[4] * p[4] && p[4] * p[4] <= dmax2);
      return m;
    }
    default:
      throw Error(MFMG_ERR_INVALID_ARG, "unknown refinement criterion");
  }
}
}  // namespace

std::vector<Cell> Octree::leaves() const {
  std::vector<Cell> out;
  for (int l = 0; l <= n_levels(); ++l) {
    if (l == 0) {
      for (int64_t k = 0; k < n0; ++k)
        for (int64_t j = 0; j < n0; ++j)
          for (int64_t i = 0; i < n0; ++i)
            if (!is_refined(0, i, j, k)) out.push_back({0, i, j, k});
      continue;
    }
    if (l - 1 >= n_levels()) break;
    for (uint64_t pk : refined[l - 1]) {
      int64_t pi, pj, pkk;
      unkey(pk, pi, pj, pkk);
      for (int c = 0; c < 8; ++c) {
        int64_t i = 2 * pi + (c & 1), j = 2 * pj + ((c >> 1) & 1), k = 2 * pkk + ((c >> 2) & 1);
        if (!is_refined(l, i, j, k)) out.push_back({l, i, j, k});
      }
    }
  }
  return out;
}

std::vector<Cell> Octree::cells_of_level(int l) const {
  std::vector<Cell> out;
  if (l == 0) {
    for (int64_t k = 0; k < n0; ++k)
      for (int64_t j = 0; j < n0; ++j)
        for (int64_t i = 0; i < n0; ++i) out.push_back({0, i, j, k});
    return out;
  }
  if (l < 1 || l - 1 >= n_levels()) return out;
  for (uint64_t pk : refined[l - 1]) {
    int64_t pi, pj, pkk;
    unkey(pk, pi, pj, pkk);
    for (int c = 0; c < 8; ++c) out.push_back({l, 2 * pi + (c & 1), 2 * pj + ((c >> 1) & 1), 2 * pkk + ((c >> 2) & 1)});
  }
  return out;
}

int64_t Octree::n_leaves() const {
  int64_t n = static_cast<int64_t>(n0) * n0 * n0;
  for (const auto& r : refined) n += 7 * static_cast<int64_t>(r.size());
  return n;
}

void Octree::add_refined(int l, std::vector<uint64_t>& keys) {
  if (keys.empty()) return;
  while (n_levels() <= l + 1) refined.emplace_back();
  auto& r = refined[l];
  r.insert(r.end(), keys.begin(), keys.end());
  sort_unique(r);
}

void Octree::refine_where(int kind, const double* params) {
  std::vector<Cell> lv = leaves();
  std::vector<std::vector<uint64_t>> add(n_levels() + 1);
  for (const Cell& c : lv)
    if (marked(*this, c.level, c.i, c.j, c.k, kind, params))
      add[c.level].push_back(cell_key(c.i, c.j, c.k));
  for (int l = 0; l < static_cast<int>(add.size()); ++l) add_refined(l, add[l]);
  close();
}

// For every refined cell P of level l >= 1 all of its 26 same-level
// neighbours inside the domain must exist, i.e. their parents be refined.
// A downward sweep suffices: refinements added at level l-1 are visited next.
void Octree::close() {
  for (int l = n_levels() - 1; l >= 1; --l) {
    if (refined[l].empty()) continue;
    std::vector<uint64_t> need;
    need.reserve(refined[l].size() * 4);
    const int64_t e = extent(l);
    for (uint64_t key : refined[l]) {
      int64_t i, j, k;
      unkey(key, i, j, k);
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            int64_t a = i + dx, b = j + dy, c = k + dz;
            if (a < 0 || b < 0 || c < 0 || a >= e || b >= e || c >= e) continue;
            uint64_t pk = cell_key(a >> 1, b >> 1, c >> 1);
            if (!std::binary_search(refined[l - 1].begin(), refined[l - 1].end(), pk)) need.push_back(pk);
          }
    }
    sort_unique(need);
    add_refined(l - 1, need);
  }
  while (n_levels() > 1 && refined.back().empty()) refined.pop_back();
}

Octree Octree::coarsened() const {
  Octree t(n0, lo, hi);
  t.refined.assign(refined.size(), {});
  for (int l = 0; l < n_levels(); ++l) {
    // keep refined cells that have at least one refined child
    std::vector<uint64_t> parents;
    if (l + 1 < n_levels()) {
      parents.reserve(refined[l + 1].size());
      for (uint64_t key : refined[l + 1]) {
        int64_t i, j, k;
        unkey(key, i, j, k);
        parents.push_back(cell_key(i >> 1, j >> 1, k >> 1));
      }
      sort_unique(parents);
    }
    std::vector<uint64_t> keep;
    std::set_intersection(refined[l].begin(), refined[l].end(), parents.begin(), parents.end(),
                          std::back_inserter(keep));
    t.refined[l] = std::move(keep);
  }
  while (t.n_levels() > 1 && t.refined.back().empty()) t.refined.pop_back();
  t.close();
  return t;
}

bool Octree::is_coarse_grid() const {
  for (const auto& r : refined)
    if (!r.empty()) return false;
  return true;
}

Octree build_octree(const mfmg_mesh_desc& d) {
  MFMG_REQUIRE(d.n0 >= 1 && d.n0 <= 64, MFMG_ERR_INVALID_ARG, "n0 must be in [1, 64]");
  MFMG_REQUIRE(d.hi > d.lo, MFMG_ERR_INVALID_ARG, "empty domain");
  MFMG_REQUIRE(d.n_global >= 0 && d.n_steps >= 0 && d.n_steps <= MFMG_MAX_STEPS, MFMG_ERR_INVALID_ARG,
               "bad refinement step counts");
  Octree t(d.n0, d.lo, d.hi);
  const double none[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int s = 0; s < d.n_global; ++s) t.refine_where(MFMG_PRED_ALL, none);
  for (int s = 0; s < d.n_steps; ++s) t.refine_where(d.kind[s], d.params[s]);
  MFMG_REQUIRE(t.n_levels() <= 18, MFMG_ERR_UNSUPPORTED, "more than 18 refinement levels");
  return t;
}

bool leaf_has_hanging(const Octree& t, const Cell& c) {
  if (c.level == 0) return false;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int nz = (dx != 0) + (dy != 0) + (dz != 0);
        if (nz == 0 || nz == 3) continue;
        int64_t a = c.i + dx, b = c.j + dy, d = c.k + dz;
        if (!t.inside(c.level, a, b, d)) continue;
        if (!t.exists(c.level, a, b, d)) return true;
      }
  return false;
}

}  // namespace mfmg
