// Degrees of freedom of a multigrid level and the per-cell data of the
// matrix-free loops (host side).
//
// Numbering.  A Q_k DoF belongs to one geometric entity of the mesh: a
// vertex, an edge (k-1 DoFs), a face ((k-1)^2) or a cell interior ((k-1)^3).
// Entities on the domain boundary carry homogeneous Dirichlet constraints and
// have no DoFs.  Entities are identified by the doubled coordinates of their
// centre on the finest lattice (unique across levels).  The DoFs of one
// entity are numbered consecutively.
//
// Cell batches (operator evaluation).  Consecutive cells along the Morton
// curve are grouped into batches whose touched DoFs fit a fixed LDS budget.
// An entity touched by one batch only is *exclusive*; otherwise *shared*.
// The global numbering puts all shared DoFs first (first-touch order over the
// batches), then the exclusive DoFs batch by batch, each batch's exclusive
// DoFs forming one contiguous range.  A batch's local vector lists its shared
// DoFs (explicit global indices) followed by its exclusive ones (a contiguous
// copy of the global range).  Cells address it with 16-bit local entity
// starts.  Shared DoFs receive one partial sum per touching batch, written
// batch by batch into a partial buffer (position = the batch's offset in the
// local shared lists plus the local index); the positions of shared DoF s are
// red_idx[red_off[s] .. red_off[s+1]-1], summed in that order by a second
// pass.
//
// Gather maps with hanging-node constraints (Section 3.2: constraints applied
// while the DoF values are set up, via an updated DoF map and in-place 1D
// interpolation).  A cell of level l >= 1 that is child (sx, sy, sz) of its
// parent can only have hanging faces and edges on the parent's outer
// boundary: the face normal to axis d on side s_d, and the edge parallel to
// axis d through the corner (s_x, s_y, s_z).  For each of the 27 entity slots
// of the cell (8 vertices, 12 edges, 6 faces, interior) the map stores the
// first DoF index of the entity, or -1 for a Dirichlet entity.  Slots lying in
// a hanging face or on a hanging edge point to the *parent's* entity of the
// same slot (the coarse neighbour's face, edge or vertex at the same relative
// position); the kernels then interpolate the gathered coarse values in place
// along the lines of the hanging faces/edges.  The mask of a cell holds
// bits 0-2 (sx, sy, sz), 3-5 (hanging face x, y, z), 6-8 (hanging edge
// x, y, z) and the cell level in bits 16-23.
#pragma once

#include <cstdint>
#include <unordered_map>
#include <vector>

#include "octree.hpp"

namespace mfmg {

enum : uint32_t {
  MASK_FACE_SHIFT = 3,
  MASK_EDGE_SHIFT = 6,
  MASK_LEVEL_SHIFT = 16,
};

constexpr int N_SLOTS = 27;

struct LevelDofs {
  int k = 1;
  int64_t n_cells = 0;
  int64_t n_dofs = 0;
  int64_t n_shared = 0;
  int64_t n_hanging_cells = 0;
  double h0 = 1.0;                // coarse-grid cell size (level-0)
  std::vector<Cell> cells;        // Morton order
  std::vector<int32_t> ent;       // [N_SLOTS][n_cells] first DoF of the slot's entity, -1 Dirichlet
  std::vector<int32_t> ent_id;    // [N_SLOTS][n_cells] entity id (-1 Dirichlet), interior included
  std::vector<uint32_t> mask;     // per cell
  std::vector<int64_t> codes;     // [n_dofs][3]
  int64_t n_entities = 0;
  // cell batches
  int64_t n_batches = 0;
  std::vector<int32_t> batch_cell_off;  // [n_batches+1]
  std::vector<int32_t> batch_sh_off;    // [n_batches+1] into sh_idx / partial buffer
  std::vector<int32_t> batch_ex_off;    // [n_batches+1] exclusive DoFs start at n_shared + batch_ex_off[b]
  std::vector<int32_t> sh_idx;          // global DoF of each local shared DoF
  std::vector<uint16_t> loc;            // [N_SLOTS][n_cells] local entity start, 0xffff Dirichlet
  std::vector<int32_t> red_off;         // [n_shared+1] CSR over the shared DoFs
  std::vector<int32_t> red_idx;         // partial-buffer positions (batch order) of each shared DoF
  // entities: key (doubled centre coordinates on the finest lattice of the
  // tree), first DoF and DoF count
  std::vector<uint64_t> ent_key;
  std::vector<int32_t> ent_first, ent_size;
  // local-smoothing levels only: per entity, lies on the refinement edge /
  // belongs to a cell that is a leaf of the tree; per DoF, the edge flag
  std::vector<uint8_t> ent_edge, ent_on_leaf, dof_edge;
  int64_t n_edge_dofs = 0;
  bool slot_hanging(int64_t c, int s) const;
};

// Scalar diffusion coefficient c(x) of the operator -div(c grad u), taken
// constant per cell.  A leaf of the finest mesh takes c at its centre; a
// refined cell (on a coarser multigrid level) the mean of its eight
// children's values, i.e. the average over the finest leaves it covers.  The
// operator uses this value rounded to bfloat16 (the form in which the cell
// mask carries it).  kind 0: c = p[0] (0 -> 1);
// kind 1: p[4] inside the ball |x - (p[0],p[1],p[2])| <= p[3], else p[5];
// kind 2: checkerboard of cubes of edge p[2] anchored at (p[3],p[3],p[3]),
// p[0] on even and p[1] on odd cubes.
struct CoefDesc {
  int kind = 0;
  double p[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double value(double x, double y, double z) const;
};
// mask bits of c rounded to the nearest bfloat16 (ties to even)
uint32_t coef_mask_bits(double c);

// Builds the DoF numbering and gather maps of `tree` at degree k; `codes`
// also computes the position codes of all DoFs.  With only_level >= 0 the
// cells are all cells of that refinement level, refined or not (a
// local-smoothing level, Section 2.1: a conforming mesh of the region they
// cover, without hanging nodes); DoFs on the boundary of that region inside
// the domain are flagged as refinement-edge DoFs.
// `coef_fine` is the finest mesh of the hierarchy (NULL: `tree`).
LevelDofs build_level_dofs(const Octree& tree, int k, bool dirichlet, bool codes = true, int only_level = -1,
                           const CoefDesc* coef = nullptr, const Octree* coef_fine = nullptr);

// Transfer data between a fine level and the next coarser one (Section 3.5).
// Geometric: every coarse cell is a fine cell (identity category) or the
// parent of 8 fine cells (refinement category).  Polynomial: same cells,
// one category.  valence[slot][fine cell] = number of transfer groups (coarse
// cells) in which the slot's entity appears unconstrained; 0 for constrained
// (hanging or Dirichlet) slots.  The prolongation weights are 1/valence.
struct TransferDofs {
  bool polynomial = false;
  std::vector<int32_t> ident_coarse, ident_fine;   // identity category pairs
  std::vector<int32_t> refined_coarse;             // refinement category coarse cells
  std::vector<int32_t> refined_fine;               // [8][n_refined] children, child c = sx + 2 sy + 4 sz
  // [N_SLOTS][n_fine_cells]: number of groups in which the entity appears
  // unconstrained (0: constrained or Dirichlet), plus TRANSFER_OWNER on the
  // one (fine cell, slot) pair that writes (prolongation) or reads
  // (restriction) the entity
  std::vector<uint8_t> valence;
  // with `coloured`: both group lists in colour order (no two groups of a
  // colour share a coarse entity) and the colour ranges
  std::vector<int64_t> ident_off, refined_off;
};

// With skip_unrefined, coarse cells that are neither fine cells nor parents of
// fine cells are left out (local-smoothing levels: the active coarse cells
// take no part in the transfer).
TransferDofs build_transfer(const LevelDofs& fine, const LevelDofs& coarse, bool polynomial,
                            bool skip_unrefined = false, bool coloured = false);

// Cells of a level colour by colour, so that no two cells of a colour share
// an entity outside their interiors (greedy in cell order, at most 64
// colours): cells[] and the colour ranges off[] (n_colours + 1).
void colour_cells(const LevelDofs& L, std::vector<int32_t>& cells, std::vector<int64_t>& off);

// Copy between the active mesh and a local-smoothing level (Algorithm 1):
// the interior (non-edge) entities of the level's leaves are entities of the
// active mesh with the same key and DoF layout; their DoFs are paired as
// (level DoF, active DoF).
struct EntityIndex {
  std::unordered_map<uint64_t, int32_t> by_key;
  explicit EntityIndex(const LevelDofs& active);
};
void ls_copy_pairs(const LevelDofs& level, const LevelDofs& active, const EntityIndex& index,
                   std::vector<int32_t>& level_dofs, std::vector<int32_t>& active_dofs);

// Dense assembled matrix of a (small) level: sum_e C_e^T A_e C_e; with
// `geo` (coarse-cell map coefficients, geometry.hpp; n0 coarse cells per
// axis) the element matrices of the mapped cells, by quadrature.
std::vector<double> assemble_dense(const LevelDofs& L, const struct Tables1D& t,
                                   const std::vector<double>* geo = nullptr, int geo_n0 = 0);

}  // namespace mfmg
