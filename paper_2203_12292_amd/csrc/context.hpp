// Library state: mesh handle and the multigrid level hierarchy on the GPU.
#pragma once

#include <memory>
#include <vector>

#include "common.hpp"
#include "dofs.hpp"
#include "geometry.hpp"
#include "kernels.hpp"
#include "octree.hpp"

struct mfmg_mesh_s {
  std::vector<mfmg::Octree> gc;  // global-coarsening sequence, index 0 = coarse grid
  int64_t n_hanging_fine = 0;
};

namespace mfmg {

struct Level {
  int mesh = 0;     // index into the global-coarsening sequence
  int only_level = -1;  // local smoothing: the refinement level whose cells form this level
  int k = 1;
  int dtype = MFMG_F64;
  int64_t n_dofs = 0, n_cells = 0, n_hanging = 0;
  DeviceArray<int32_t> ent, ijk;
  std::vector<int32_t> host_levels, host_ijk;  // cell order of the level
  DeviceArray<uint32_t> mask;
  DeviceArray<CellMeta> meta;
  DeviceArray<int32_t> batch_cell, batch_sh, batch_ex, sh_idx, red_off, red_idx;
  DeviceArray<char> partial;
  CellView view;
  DeviceArray<double> diag;
  DeviceArray<char> dinv;  // 1/diag in the level's arithmetic type
  double lmin = 0.0, lmax = 1.0;
  // work vectors (max_rhs interleaved): storage type and arithmetic type
  DeviceArray<char> x, b, r, d, t, tmp_cast;
  // deterministic mode: the level's cells colour by colour (diagonal, load
  // vector) and the colour ranges of the transfer groups (restriction)
  DeviceArray<int32_t> color_cells;
  std::vector<int64_t> color_off, tr_ident_off, tr_refined_off;
  // transfer from level l-1 (fine side = this level)
  bool has_transfer = false;
  DeviceArray<int32_t> tr_ident_c, tr_ident_f, tr_ref_c, tr_ref_f;
  DeviceArray<uint8_t> tr_valence;
  TransferView tview;
  // local smoothing: refinement-edge DoFs, and the copy to / from the active
  // mesh (level DoF cp_level[q] <-> active DoF cp_active[q])
  int64_t n_edge = 0, n_copy = 0;
  std::vector<uint8_t> host_edge;
  DeviceArray<int32_t> edge_idx, cp_level, cp_active;
};

struct NetState {
  int nq = 0, n_cells = 0, n0 = 0, n_params = 0;
  DeviceArray<int32_t> node_dof;  // [n_cells][nq] coarse DoF of each cell node, -1 Dirichlet
  DeviceArray<float> inv_val;     // 1 / number of coarse cells containing the DoF
  DeviceArray<float> centre;      // [n_cells][3]
  DeviceArray<float> params;
  DeviceArray<double> work;
  DeviceArray<int> counters;      // accepted, rejected
  DeviceArray<double> relsum;     // sum of ||b0 - A0 y|| / ||b0|| of the predictions
  int mode = MFMG_COARSE_EXACT;
  double tau = 0.5;
  // recording of coarse right-hand sides
  int rec_capacity = 0, rec_count = 0;
  DeviceArray<double> record;
  // training buffers
  DeviceArray<float> X, T, z1, h1, z2, h2, y, d3, d2, d1, lossbuf;
};

// V-cycles of the outer solver replayed from HIP graphs, one per (x, b,
// n_vec); captured on a private stream of default priority.
struct GraphCache {
  struct Entry {
    const void* x;
    const void* b;
    int nv;
    hipGraphExec_t exec;
  };
  struct Key {
    const void* x;
    const void* b;
    int nv;
    bool operator==(const Key& o) const { return x == o.x && b == o.b && nv == o.nv; }
  };
  std::vector<Entry> entries;
  std::vector<Key> seen;  // (x, b, n_vec) run eagerly once
  hipStream_t capture = nullptr;
  GraphCache() = default;
  GraphCache(const GraphCache&) = delete;
  GraphCache& operator=(const GraphCache&) = delete;
  ~GraphCache() {
    clear();
    if (capture) (void)hipStreamDestroy(capture);
  }
  // forget every captured cycle (their kernel arguments are out of date)
  void clear() {
    for (auto& e : entries) (void)hipGraphExecDestroy(e.exec);
    entries.clear();
    seen.clear();
  }
};

struct Context {
  mfmg_level_desc desc{};
  GraphCache graphs;
  CoefDesc coef;  // diffusion coefficient (constant per cell)
  GeoDesc geo;    // cell geometry; kind 0: axis-aligned cubes
  std::vector<double> geo_host;            // coarse-cell map coefficients [n0^3][24]
  DeviceArray<double> geo64;
  DeviceArray<float> geo32;
  int geo_n0 = 0;
  std::vector<Octree> meshes;
  std::vector<Level> levels;  // 0 = coarsest
  // local smoothing: `levels` are the refinement levels and `active` is the
  // operator of the leaves (the mesh the outer solver works on)
  bool ls = false;
  Level active;
  int max_rhs = 1;
  int cheb_degree = 3;
  // exact coarse solver: dense inverse of A^(0), and the host description of
  // level 0 it is assembled from (kept to reassemble it)
  int64_t n0 = 0;
  LevelDofs coarse_host;
  DeviceArray<double> coarse_inv64;
  DeviceArray<double> coarse_A64;
  NetState net;
  DeviceArray<float> coarse_inv32;
  // parameters of the load vector (mfmg_rhs), staged from the host; grown
  // only when a call needs more than any call before
  DeviceArray<double> rhs_params;
  // FP64 CG work space on the finest level
  DeviceArray<double> cg_r, cg_p, cg_q, cg_z, cg_zold, cg_partial, cg_scalar;
  std::vector<double> host_scalar;
  hipStream_t stream = nullptr;

  Level& fine() { return ls ? active : levels.back(); }
  // level -1 addresses the active mesh
  Level& level(int l) {
    if (l == MFMG_LEVEL_ACTIVE) return fine();
    MFMG_REQUIRE(l >= 0 && l < static_cast<int>(levels.size()), MFMG_ERR_INVALID_ARG, "level out of range");
    return levels[l];
  }
};

void setup_context(Context& ctx, const mfmg_mesh_s& mesh, const mfmg_level_desc& desc, hipStream_t s);

// operations on levels (all asynchronous on `s` unless noted)
void level_vmult(Context& ctx, int l, int dtype, int nv, void* dst_acc, const void* src, hipStream_t s);
void level_smooth(Context& ctx, int l, int nv, void* x, const void* b, bool x_is_zero, double lmin, double lmax,
                  hipStream_t s);
void level_residual(Context& ctx, int l, int nv, void* r, const void* b, const void* x, hipStream_t s);
void level_prolongate_add(Context& ctx, int fine, int dtype, int nv, void* dst, const void* src, hipStream_t s);
void level_restrict_add(Context& ctx, int fine, int dtype, int nv, void* dst, const void* src, hipStream_t s);
void coarse_solve(Context& ctx, int dtype, int nv, void* x, const void* b, hipStream_t s);
void vcycle(Context& ctx, int nv, double* x, const double* b, hipStream_t s);
void fmg(Context& ctx, int nv, double* x, const double* b, int cycles, hipStream_t s);
void copy_to_mg(Context& ctx, int l, int nv, void* dst, const double* src, hipStream_t s);
void copy_from_mg(Context& ctx, int l, int nv, double* dst, const void* src, hipStream_t s);
int pcg(Context& ctx, int nv, double* x, const double* b, double rtol, int max_it, bool flexible,
        mfmg_solve_stats* stats, hipStream_t s);
// new cellwise-constant coefficient from the finest level's cell values
// (device array); synchronizes `s`
void set_coefficient(Context& ctx, const double* c_fine, hipStream_t s);

}  // namespace mfmg
