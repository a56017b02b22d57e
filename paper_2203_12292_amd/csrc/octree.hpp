// Octree forest over an n0^3 coarse grid (host side).
//
// Cells of level l are integer triples (i, j, k), 0 <= i, j, k < n0 * 2^l.
// The tree is the set of refined cells per level (sorted 63-bit keys).  A cell
// exists when its parent is refined (all level-0 cells exist); a leaf exists
// and is not refined.  Meshes are built by the refinement criteria of the
// paper's test cases (Section 4 "Examples"), each step followed by the
// one-irregularity closure; global coarsening (Section 2.2) removes all
// terminal families at once and closes again.
#pragma once

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/mfmg.h"

namespace mfmg {

struct Cell {
  int level;
  int64_t i, j, k;
};

inline uint64_t cell_key(int64_t i, int64_t j, int64_t k) {
  return (static_cast<uint64_t>(i) << 42) | (static_cast<uint64_t>(j) << 21) | static_cast<uint64_t>(k);
}

class Octree {
 public:
  int n0 = 1;
  double lo = 0.0, hi = 1.0;
  std::vector<std::vector<uint64_t>> refined;  // per level, sorted unique

  Octree() = default;
  Octree(int n0_, double lo_, double hi_) : n0(n0_), lo(lo_), hi(hi_) { refined.resize(1); }

  int n_levels() const { return static_cast<int>(refined.size()); }
  int64_t extent(int l) const { return static_cast<int64_t>(n0) << l; }
  double h(int l) const { return (hi - lo) / (n0 * std::ldexp(1.0, l)); }

  bool is_refined(int l, int64_t i, int64_t j, int64_t k) const {
    if (l < 0 || l >= n_levels()) return false;
    const auto& r = refined[l];
    return std::binary_search(r.begin(), r.end(), cell_key(i, j, k));
  }
  bool inside(int l, int64_t i, int64_t j, int64_t k) const {
    int64_t e = extent(l);
    return i >= 0 && j >= 0 && k >= 0 && i < e && j < e && k < e;
  }
  bool exists(int l, int64_t i, int64_t j, int64_t k) const {
    if (!inside(l, i, j, k)) return false;
    if (l == 0) return true;
    return is_refined(l - 1, i >> 1, j >> 1, k >> 1);
  }
  bool is_leaf(int l, int64_t i, int64_t j, int64_t k) const {
    return exists(l, i, j, k) && !is_refined(l, i, j, k);
  }

  // leaves of every level
  std::vector<Cell> leaves() const;
  // every cell of level l, refined or not
  std::vector<Cell> cells_of_level(int l) const;
  int64_t n_leaves() const;

  void refine_where(int kind, const double* params);
  void close();
  Octree coarsened() const;
  bool is_coarse_grid() const;

 private:
  void add_refined(int l, std::vector<uint64_t>& keys);
};

Octree build_octree(const mfmg_mesh_desc& d);

// A leaf of level l >= 1 carries hanging-node constraints when one of the 18
// level-l cells sharing a face or an edge with it lies in the domain but does
// not exist.
bool leaf_has_hanging(const Octree& t, const Cell& c);

}  // namespace mfmg
