/*
 * mfmg — matrix-free multigrid on locally refined hexahedral meshes, MI355X.
 *
 * C ABI of the hot path of the solver described in
 *   M. Munch, T. Heister, L. Prieto Saavedra, M. Kronbichler,
 *   "Efficient distributed matrix-free multigrid methods on locally refined
 *    meshes for FEM computations", arXiv 2203.12292.
 *
 * Problem: -Laplace(u) = f on a cube, u = 0 on its boundary, continuous Q_k
 * Lagrange elements (Gauss-Lobatto nodes, Gauss quadrature with (k+1)^3
 * points) on an octree mesh whose touching leaves differ by at most one level.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Return value: MFMG_OK (0) or a negative MFMG_ERR_* code; the message of
 *    the last error of the calling thread is returned by mfmg_last_error().
 *    Invalid handles, levels, dtypes, degrees or null pointers give
 *    MFMG_ERR_INVALID_ARG / MFMG_ERR_UNSUPPORTED and change nothing.
 *  - Vectors hold the *free* DoFs of a level only (Dirichlet and hanging-node
 *    DoFs are constraints, Section 3.1, not unknowns).  With n_vec > 1 the
 *    layout is DoF-major interleaved: entry (i, v) at index i*n_vec + v.
 *  - Vector arguments are device pointers (hipMalloc'd or torch CUDA/HIP
 *    tensors), contiguous, owned by the caller, of the element type named by
 *    the dtype argument (double, float, or bfloat16 as uint16 bits).
 *  - `stream` is a hipStream_t (NULL = default stream).  Calls marked
 *    [async] only enqueue work on it; the others synchronise it.
 *  - The library owns mesh and level data; it allocates device memory in
 *    mfmg_setup_levels (metadata, per-level work vectors) and frees it in
 *    mfmg_destroy_ctx.  The calls below allocate nothing else, except the
 *    learned correction's recording and training (mfmg_net_record,
 *    mfmg_net_loss_grad, mfmg_net_train) and mfmg_rhs when its parameters
 *    exceed 8 Gaussians per vector (the staging buffer then grows once).
 */
#ifndef MFMG_H
#define MFMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mfmg_mesh_s* mfmg_mesh;
typedef struct mfmg_ctx_s* mfmg_ctx;

enum {
  MFMG_OK = 0,
  MFMG_ERR_INVALID_ARG = -1,
  MFMG_ERR_UNSUPPORTED = -2,
  MFMG_ERR_HIP = -3,
  MFMG_ERR_OOM = -4,
  MFMG_ERR_NOT_CONVERGED = -5,
  MFMG_ERR_BREAKDOWN = -6,
  MFMG_ERR_NET_REJECTED = -7 /* informational: learned correction rejected, fallback used */
};

typedef enum { MFMG_F64 = 0, MFMG_F32 = 1, MFMG_BF16 = 2 } mfmg_dtype;

/* Refinement criteria of the test meshes (Section 4, "Examples"); c = cell
 * centre.  ALL: every cell.  BALL (x0,y0,z0,r): |c-x0|^2 <= r^2.
 * BOX_LE (a,b,c): c <= (a,b,c) componentwise (the paper's octant).
 * BAND (x0,y0,z0,r1,r2): r1^2 <= |c-x0|^2 <= r2^2 (the paper's shell).
 * SPHERE_CUT (x0,y0,z0,ra,rb): the closed cell box meets the sphere of radius
 * ra (or rb, if rb > 0) about x0. */
enum { MFMG_PRED_ALL = 0, MFMG_PRED_BALL = 1, MFMG_PRED_BOX_LE = 2, MFMG_PRED_BAND = 3,
       MFMG_PRED_SPHERE_CUT = 4 };

#define MFMG_MAX_STEPS 16
#define MFMG_MAX_LEVELS 32

typedef struct {
  int n0;          /* coarse grid n0^3 cubes */
  double lo, hi;   /* domain [lo, hi]^3 */
  int n_global;    /* uniform refinements first */
  int n_steps;     /* then one refinement per step, each followed by closure */
  int kind[MFMG_MAX_STEPS];
  double params[MFMG_MAX_STEPS][8];
} mfmg_mesh_desc;

/* Level sequences (coarse to fine):
 *  H        geometric global coarsening at the fine degree (Section 2.2);
 *  P_THEN_H polynomial coarsening p_c = floor(p_f/2) on the fine mesh
 *           (Section 2.3), then geometric global coarsening at degree 1;
 *  H_THEN_P geometric global coarsening at the fine degree, then polynomial
 *           coarsening on the coarse grid (keeps the coarse problem small). */
/*  LS       geometric local smoothing (Section 2.1): level l holds every
 *           cell of refinement level l, refined or not (no hanging nodes);
 *           DoFs where such a level ends inside the domain form the
 *           refinement edge.  The V-cycle follows the local-smoothing branch
 *           of Algorithm 2 and the copy to and from the levels of
 *           Algorithm 1; the outer solver works on the leaves (the active
 *           mesh, level index MFMG_LEVEL_ACTIVE).  Needs dirichlet = 1 and
 *           one storage type for all levels.
 *  LS_THEN_P local smoothing down to the coarse grid, then polynomial
 *           coarsening on the coarse grid (levels 0 .. P-1 have degrees
 *           1, 2, ..., floor(k/2); they cover the domain, have no edge and
 *           receive no copied right-hand side).
 *  HP       geometric and polynomial global coarsening in one step (the
 *           option the paper's outlook names): each level coarsens the
 *           mesh once and halves the degree, while both are possible;
 *           then the remaining one alone.  The transfer of such a step
 *           interpolates the coarse degree-k/2 function of a parent cell
 *           at the degree-k nodes of its children. */
enum { MFMG_SCHEME_H = 0, MFMG_SCHEME_P_THEN_H = 1, MFMG_SCHEME_H_THEN_P = 2, MFMG_SCHEME_LS = 3,
       MFMG_SCHEME_LS_THEN_P = 4, MFMG_SCHEME_HP = 5 };

/* Level index of the active mesh (the leaves) in every call that takes a
 * level: the finest level under global coarsening, the operator of the leaves
 * with its hanging-node constraints under local smoothing. */
#define MFMG_LEVEL_ACTIVE (-1)

typedef struct {
  int degree;            /* finest degree k, 1 <= k <= 6 */
  int scheme;            /* MFMG_SCHEME_* */
  int dirichlet;         /* 1: homogeneous Dirichlet on the whole boundary;
                            0: none (pure Neumann): the operator is singular
                            (constants are its null space), so only the
                            level calls (vmult, diagonal, smooth, residual,
                            transfers, rhs, distribute) are available and
                            coarse_solve, vcycle and solve return
                            MFMG_ERR_UNSUPPORTED */
  int n_level_dtype;     /* entries used in level_dtype (0: all MFMG_F64) */
  int level_dtype[MFMG_MAX_LEVELS]; /* storage type of V-cycle level vectors,
                                       index 0 = coarsest; missing = last entry */
  int cheb_degree;       /* Chebyshev degree (paper: 3), 0 -> 3 */
  double smoothing_range;/* lambda_min = lambda_max / range, 0 -> 20 */
  double eig_safety;     /* lambda_max = safety * estimate, 0 -> 1.2 */
  int eig_iterations;    /* CG-Lanczos steps for the estimate, 0 -> 15 */
  int max_rhs;           /* largest n_vec of vcycle/solve, 0 -> 1 (max 8) */
  int drop_coarse;       /* global-coarsening schemes: leave out this many of
                            the coarsest levels, so that the exact coarse
                            solver acts on a finer level, possibly one with
                            hanging nodes (the early switch of the paper's
                            outlook); 0 = none.  The new coarsest level must
                            have at most 12000 DoFs. */
  int coef_kind;         /* diffusion coefficient c of -div(c grad u), constant
                            per cell and rounded to bfloat16: a leaf of the
                            finest mesh takes c at its centre, a refined cell
                            of a coarser level the mean of its 8 children's
                            values (the average over the finest leaves it
                            covers).  With p = coef_params:
                            0: c = p[0] (0 -> 1);
                            1: p[4] inside the ball |x - p[0..2]| <= p[3],
                               else p[5];
                            2: checkerboard of cubes of edge p[2] anchored
                               at (p[3],p[3],p[3]), p[0] on even and p[1]
                               on odd cubes.
                            c must lie in [1e-30, 1e30].  The load vector
                            (mfmg_rhs) does not depend on c. */
  double coef_params[8];
  int graph_vcycle;      /* 1: mfmg_solve replays its V-cycles from a HIP graph
                            (captured once per vector pair on a private
                            stream after a first eager cycle; fewer launches
                            for small levels).  The learned coarse
                            correction and the recording of coarse
                            right-hand sides keep the eager path.  0 = eager. */
  int fmg_start;         /* 1: mfmg_solve starts from one full-multigrid pass
                            (mfmg_fmg, one V-cycle per level) instead of
                            x0 = 0; the stopping rule stays relative to
                            ||b||.  Global-coarsening schemes only. */
  int geom_kind;         /* cell geometry (Section 3.2: the quadrature-point
                            operation with the Jacobian J = dx/dxi of each
                            cell map).  The vertices of the coarse grid are
                            moved; each coarse cell becomes the trilinear
                            image of the cube through its moved vertices and
                            its descendants inherit that map, so the levels
                            stay nested.  With p = geom_params:
                            0: none (axis-aligned cubes, the Kronecker form
                               of the cell operator);
                            1: affine, x' = M x with
                               M = [[p0,p1,p2],[0,p3,p4],[0,0,p5]];
                            2: interior bump, x' = x + p0 s(x) (p1,p2,p3),
                               s(x) = prod_d sin(pi (x_d - lo)/(hi - lo))
                               (the domain boundary stays in place).
                            Kinds 1-2 use the general operator (values and
                            reference gradients at the Gauss points, the
                            metric term w |det J| J^-1 J^-T computed per
                            point from 24 numbers per coarse cell), and the
                            load vector integrates over the mapped cells.
                            Global-coarsening schemes only; every cell map
                            must keep det J > 0. */
  double geom_params[8];
  int deterministic;     /* 1: repeated calls give bitwise identical results
                            (for debugging; slower).  The operator adds its
                            cells' contributions to a batch in cell order,
                            one cell at a time, and sums the DoFs shared
                            between batches from per-batch partial sums in
                            a fixed order; the restriction, the diagonal
                            and the load vector run colour by colour (no
                            two cells or transfer groups of a colour share
                            an entity) with plain adds instead of atomics.
                            Everything else on the solve path
                            (prolongation, dot products, coarse solve) has
                            a fixed order anyway.  Not covered: the learned
                            correction's inference and training.  0:
                            atomics (default). */
} mfmg_level_desc;

typedef struct {
  int iterations;
  int converged;
  double initial_residual;   /* ||b||_2 */
  double final_residual;     /* ||b - A x||_2 / ||b||_2 (worst over vectors) */
  double residual_history[256];
  double time_ms;            /* solve time, set-up excluded */
  int coarse_fallbacks;      /* learned correction rejected -> exact solve */
  int coarse_accepted;       /* learned correction accepted */
} mfmg_solve_stats;

/* ---- set-up (host; synchronous) ----------------------------------------- */

/* Builds the mesh (refinement + one-irregularity closure, Section 4) and its
 * global-coarsening sequence (Section 2.2): all terminal families are
 * coarsened at once and the closure re-applied until the coarse grid is left.
 * *out is owned by the caller until mfmg_destroy_mesh. */
int mfmg_setup_mesh(const mfmg_mesh_desc* desc, mfmg_mesh* out);

/* Number of global-coarsening meshes (>= 1) and the leaf count of each,
 * index 0 = coarse grid; cells may be NULL.  n_hanging_cells (optional) gets
 * the number of leaves of the finest mesh with hanging-node constraints. */
int mfmg_mesh_info(mfmg_mesh mesh, int* n_meshes, int64_t* cells, int64_t* n_hanging_cells);

/* Builds the multigrid levels on the GPU: DoF numbering, per-cell gather maps
 * with hanging-node masks (Section 3.2, constraints applied in the gather),
 * transfer categories and valence weights (Section 3.5), the diagonal
 * (Eq. impl:mf:diagonal), Chebyshev intervals and the exact coarse solver.
 * The mesh handle may be destroyed afterwards. */
int mfmg_setup_levels(mfmg_mesh mesh, const mfmg_level_desc* desc, void* stream, mfmg_ctx* out);

int mfmg_n_levels(mfmg_ctx ctx, int* n_levels);

/* level: 0 = coarsest, MFMG_LEVEL_ACTIVE = the active mesh.  Any output
 * pointer may be NULL. */
int mfmg_level_info(mfmg_ctx ctx, int level, int64_t* n_dofs, int64_t* n_cells, int* degree,
                    int* dtype, int64_t* n_hanging_cells);

/* Exact position code of every free DoF (host array [n_dofs][3]).  Per axis:
 * a lattice point of the level-20 lattice P (cell vertices, and the middle
 * Gauss-Lobatto node of an interval for even k) is coded 2P; the a-th node of
 * interval i of level l otherwise is 2*(((l<<25)+i)*16+a)+1.  Equal codes mean
 * the same point; used to match DoFs with an independent implementation. */
int mfmg_level_dof_codes(mfmg_ctx ctx, int level, int64_t* codes);

/* Smoother interval [lambda_min, lambda_max] of D^{-1}A used by level l. */
int mfmg_smoother_range(mfmg_ctx ctx, int level, double* lambda_min, double* lambda_max);

/* Host-only inspection (no GPU needed): DoF numbering of global-coarsening
 * mesh `mesh_index` (0 = coarse grid) at degree k, and the assembled matrix
 * sum_e C_e^T A_e C_e built from the same per-cell gather maps and hanging-node
 * line rules the kernels use.  Call with codes = dense = NULL to get *n_dofs;
 * then codes ([n_dofs][3], as mfmg_level_dof_codes) and/or dense
 * ([n_dofs][n_dofs] row-major, only for n_dofs <= 20000) are filled. */
int mfmg_host_level_matrix(mfmg_mesh mesh, int mesh_index, int degree, int dirichlet, int64_t* n_dofs,
                           int64_t* codes, double* dense);

/* Host-only inspection of a local-smoothing level (Section 2.1): all cells of
 * refinement level `level` of the finest mesh at degree k, Dirichlet
 * boundary.  Call with every array NULL to get *n_dofs and *n_copy; then
 * codes ([n_dofs][3]), edge (one byte per DoF, 1 = refinement edge), dense
 * (the assembled level matrix incl. edge rows, n_dofs <= 20000) and the copy
 * map of Algorithm 1 (copy_level[q] <-> copy_active[q], active DoFs numbered
 * as by mfmg_host_level_matrix on the finest mesh) may be filled. */
int mfmg_host_ls_level(mfmg_mesh mesh, int level, int degree, int64_t* n_dofs, int64_t* n_copy,
                       int64_t* codes, uint8_t* edge, double* dense, int32_t* copy_level,
                       int32_t* copy_active);

/* ---- hot path (device; [async] on `stream`) ----------------------------- */

/* [async] dst = A^(l) src, Eq. (impl:mf): per cell gather G_e with the
 * hanging-node constraints C_e applied in registers/LDS by 1D interpolation,
 * sum-factorised evaluation S_e, quadrature-point scaling Q_e, transposed
 * steps, constrained scatter-add.  dst and src must not alias. */
int mfmg_vmult(mfmg_ctx ctx, int level, int dtype, int n_vec, void* dst, const void* src,
               void* stream);

/* [async] dst = A^(l) src as mfmg_vmult (same kernels, same result), for
 * callers that cannot allocate memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  Allocates nothing: the
 * operator's work space (the partial sums of the DoFs shared between cell
 * batches, and for MFMG_BF16 the FP32 result before rounding) lives in one
 * fixed device array of 64 MiB per GPU, held by the library until the
 * process ends.  A level whose work space exceeds it
 * (sizeof(arithmetic type) x n_vec x shared entries, + 4 x n_vec x n_dofs
 * for MFMG_BF16) is refused with MFMG_ERR_UNSUPPORTED before any work.  All
 * calls on one GPU share that array: two calls that overlap in time on one
 * GPU (different streams, or threads) race and give wrong results; calls
 * ordered on one stream are safe. */
int mfmg_vmult_noalloc(mfmg_ctx ctx, int level, int dtype, int n_vec, void* dst, const void* src,
                       void* stream);

/* [async] diag = diagonal of A^(l) (Eq. impl:mf:diagonal, unit-vector
 * applications per cell with C_e applied from both sides). */
int mfmg_diagonal(mfmg_ctx ctx, int level, int dtype, void* diag, void* stream);

/* [async] Chebyshev smoothing of degree cheb_degree around point Jacobi
 * (Section 3.3) of A^(l) x = b; x_is_zero: start from x = 0 (skips one
 * operator evaluation).  lambda: NULL for the set-up interval, else
 * {lambda_min, lambda_max}.  Uses the level's internal work vectors. */
int mfmg_smooth(mfmg_ctx ctx, int level, int dtype, int n_vec, void* x, const void* b,
                int x_is_zero, const double* lambda, void* stream);

/* [async] r = b - A^(l) x (Algorithm 2, residual step). */
int mfmg_residual(mfmg_ctx ctx, int level, int dtype, int n_vec, void* r, const void* b,
                  const void* x, void* stream);

/* [async] dst_fine += P src_coarse between level fine_level-1 and fine_level
 * (Eq. eq:impl:loop:categorized: coarse gather with constraints, category
 * prolongation, valence weights W, scatter). */
int mfmg_prolongate_add(mfmg_ctx ctx, int fine_level, int dtype, int n_vec, void* dst_fine,
                        const void* src_coarse, void* stream);

/* [async] dst_coarse += P^T src_fine (restriction = transposed prolongation). */
int mfmg_restrict_add(mfmg_ctx ctx, int fine_level, int dtype, int n_vec, void* dst_coarse,
                      const void* src_fine, void* stream);

/* [async] x = A^(0)^{-1} b on the coarsest level (exact: dense inverse from a
 * host Cholesky factorisation of the assembled coarse matrix).
 *
 * Every vector argument of the level calls may be NULL when its level has no
 * free DoF (for example one Q1 cell with Dirichlet boundary); such a call
 * does nothing. */
int mfmg_coarse_solve(mfmg_ctx ctx, int dtype, int n_vec, void* x, const void* b, void* stream);

/* [async] Algorithm 1: copy b (FP64, active mesh) to the levels in their
 * storage type, one V-cycle (Algorithm 2: global-coarsening branch, or the
 * local-smoothing branch under MFMG_SCHEME_LS), copy x back to FP64.
 * n_vec <= max_rhs. */
int mfmg_vcycle(mfmg_ctx ctx, int n_vec, void* x_f64, const void* b_f64, void* stream);

/* [async] Full multigrid (textbook FMG with V-cycles; the paper names it as a
 * solver that global coarsening makes easy to build, Section 2.2): b (FP64,
 * finest level) is restricted to every level, b^(l-1) = P^T b^(l); the
 * coarsest level is solved exactly; on each finer level the prolongated
 * coarser result is the initial guess of `cycles` V-cycles (Algorithm 2,
 * presmoothing from that guess).  x (FP64) receives the finest result.
 * Global-coarsening schemes only (MFMG_ERR_UNSUPPORTED under local
 * smoothing); 1 <= cycles <= 16; n_vec <= max_rhs.  Uses the levels' work
 * vectors, like mfmg_vcycle. */
int mfmg_fmg(mfmg_ctx ctx, int n_vec, void* x_f64, const void* b_f64, int cycles, void* stream);

/* [async] Algorithm 1, copy to the levels, for level l: dst (level storage
 * type, [n_dofs(l)][n_vec]) is zeroed, then receives the values of the
 * active-mesh vector src (FP64) at the active DoFs that belong to level l.
 * Under global coarsening l must be the finest level and dst = src (cast).
 * Under local smoothing an active DoF belongs to the coarsest level among
 * the leaves that have it as a node, where it is an interior (non-edge) DoF;
 * every active DoF belongs to exactly one level. */
int mfmg_copy_to_mg(mfmg_ctx ctx, int level, int n_vec, void* dst, const void* src_f64, void* stream);

/* [async] Algorithm 1, copy from the levels: the active DoFs that belong to
 * level l (as in mfmg_copy_to_mg) receive their values from src (level
 * storage type); the other entries of dst (FP64) are left unchanged. */
int mfmg_copy_from_mg(mfmg_ctx ctx, int level, int n_vec, void* dst_f64, const void* src, void* stream);

/* Refinement-edge DoFs of level l (Section 2.1, local smoothing): their
 * number in *n_edge and, if flags is not NULL, one byte per DoF (host array
 * [n_dofs(l)], 1 = edge).  Smoothing treats them as Dirichlet values (their
 * inverse diagonal is 0, so A_SS acts on the interior DoFs and the smoother
 * keeps x_E); the residual step gives -A_ES x_S on them, and after the
 * prolongation the smoother's operator applies A_SE x_E, i.e. the modified
 * right-hand side b_S - A_SE x_E of the edge step.  0 under global
 * coarsening. */
int mfmg_level_edge(mfmg_ctx ctx, int level, int64_t* n_edge, uint8_t* flags);

/* FP64 conjugate gradients preconditioned by one V-cycle per iteration
 * (Section 2), x0 = 0, stopped when ||b - A x||_2 <= rtol ||b||_2 for every
 * vector (n_vec vectors in lock step).  flexible = 1 uses the Polak-Ribiere
 * beta (needed when the preconditioner is not a fixed linear operator).
 * Returns MFMG_ERR_NOT_CONVERGED after max_it iterations (x holds the last
 * iterate), MFMG_ERR_BREAKDOWN if p^T A p <= 0.  Synchronous. */
int mfmg_solve(mfmg_ctx ctx, int n_vec, void* x_f64, const void* b_f64, double rtol, int max_it,
               int flexible, mfmg_solve_stats* stats, void* stream);

/* Load vector b_i = int f phi_i (Gauss (k+1)^3 points, constraints
 * applied, Dirichlet rows 0) on level l in FP64.  kind 0: f = params[0];
 * kind 1: f = sum of n_terms Gaussians a exp(-|x-c|^2/(2w^2)), rows
 * (cx,cy,cz,w,a) in params (host memory), n_terms rows per vector;
 * kind 2: f = params[0] sin(params[1] x) sin(params[1] y) sin(params[1] z)
 * (manufactured solutions).
 * Synchronises `stream` (params are staged through device memory). */
enum { MFMG_RHS_CONST = 0, MFMG_RHS_GAUSS = 1, MFMG_RHS_SINE = 2 };
int mfmg_rhs(mfmg_ctx ctx, int level, int kind, const double* params, int n_terms, int n_vec,
             void* b_f64, void* stream);

/* [async] Constraint distribution (Section 3.1): the values of the FE
 * function x (free DoFs, FP64) at every node of every cell, hanging nodes
 * interpolated from their constraining DoFs and Dirichlet nodes 0.  out is
 * [n_cells][(k+1)^3] (nodes lexicographic, x fastest) in the level's cell
 * order; cell coordinates via mfmg_level_cells. */
int mfmg_distribute(mfmg_ctx ctx, int level, const void* x_f64, void* out_f64, void* stream);

/* Cells of a level in the library's order: levels[c] and ijk[3c..3c+2]
 * (host arrays of n_cells and 3 n_cells entries). */
int mfmg_level_cells(mfmg_ctx ctx, int level, int32_t* levels, int32_t* ijk);

/* New diffusion coefficient, transferred to every multigrid level on the
 * device (the interpolate_to_mg step of the transfer class, Section 3.5, for
 * a field that is constant per cell; the operator -div(c grad u) of
 * Eq. (impl:mf) with c in the quadrature-point term).  c_f64: device array of
 * one value per cell of the finest level, in the order of
 * mfmg_level_cells(ctx, n_levels - 1), each in [1e-30, 1e30] (else
 * MFMG_ERR_INVALID_ARG and nothing changes).  Each coarser level's cell takes
 * the value of the same cell on the next finer level or the mean of its
 * eight children (summed in child order, x fastest), i.e. the average over
 * the finest cells it covers, as at set-up; the operator uses it rounded to
 * bfloat16.  The diagonals, the Chebyshev intervals (eigenvalue estimate
 * repeated), the dense coarse inverse (reassembled on the host from the
 * coarse level's cells) and the learned correction's residual check follow;
 * V-cycles captured in graphs are dropped.  The network keeps its
 * parameters.  Set-up call: allocates temporary device memory and
 * synchronizes the stream.  Local-smoothing schemes: MFMG_ERR_UNSUPPORTED. */
int mfmg_set_coefficient(mfmg_ctx ctx, const void* c_f64, void* stream);

/* ---- learned coarse correction (an extension, not in the paper) ---------
 * A per-coarse-cell network replaces the exact coarse solve at level 0: input
 * the coarse right-hand side at the cell's (k+1)^3 nodes divided by
 * s = ||b0||_2 and the cell centre; two hidden layers of width 64 (GELU);
 * output the cell's nodal correction divided by s; nodes of several cells
 * average their cells' outputs.  The exact coarse operator checks every
 * prediction: if ||b0 - A0 y||_2 > tau ||b0||_2 the exact solution is used.
 * Flat FP32 parameters: W1 ((nq+3) x 64, row-major), b1, W2 (64x64), b2,
 * W3 (64 x nq), b3, nq = (k+1)^3 of level 0.  Requires a coarse level
 * without hanging nodes, at most 2048 DoFs and nq + 3 <= 64 (degree <= 2);
 * otherwise every mfmg_net_* call except mfmg_net_mode(EXACT) returns
 * MFMG_ERR_UNSUPPORTED. */
enum { MFMG_COARSE_EXACT = 0, MFMG_COARSE_LEARNED = 1, MFMG_COARSE_ZERO = 2 };

typedef struct {
  int epochs;           /* passes over the data set */
  int batch_rows;       /* rows (pairs x coarse cells) per Adam step, 0 -> 4096 */
  double lr;            /* Adam step size, 0 -> 1e-3 (beta1 0.9, beta2 0.999, eps 1e-8) */
  uint64_t init_seed;   /* != 0: re-initialise parameters (He normal) from this seed */
  uint64_t shuffle_seed;/* row order of the epochs */
} mfmg_net_train_desc;

int mfmg_net_n_params(mfmg_ctx ctx, int* n);
/* Record the right-hand side reaching the coarse solver in every following
 * V-cycle (up to `capacity` of them; 0 stops and frees). Synchronous. */
int mfmg_net_record(mfmg_ctx ctx, int capacity);
int mfmg_net_n_recorded(mfmg_ctx ctx, int* n);
/* Copy parameters from/to host memory (n = mfmg_net_n_params). */
int mfmg_net_set_params(mfmg_ctx ctx, const float* theta, int n);
int mfmg_net_get_params(mfmg_ctx ctx, float* theta, int n);
/* Mean squared error and its gradient (device FP32 arrays) over n_rows rows
 * X [n_rows][nq+3], T [n_rows][nq] with the current parameters.  Synchronous. */
int mfmg_net_loss_grad(mfmg_ctx ctx, int n_rows, const float* X, const float* T, float* grad, float* loss);
/* Train on the recorded pairs (b0, A0^{-1} b0) with Adam on the GPU;
 * history (host, `epochs` floats, may be NULL) gets the data-set loss after
 * each epoch.  Synchronous. */
int mfmg_net_train(mfmg_ctx ctx, const mfmg_net_train_desc* desc, float* history);
/* [async] y = the network's coarse correction for the level-0 right-hand
 * side b, without the residual check: per coarse cell, the MLP maps
 * (b at the cell's nodes / s, cell centre) to nodal values; y_i is s times the
 * mean of the values of the cells that have DoF i as a node, s = ||b||_2
 * (y = 0 for b = 0).  b and y are level-0 vectors of `dtype` (the level's
 * storage type or any other), n0 entries each, caller-owned device memory;
 * the network arithmetic is FP32, the averaging FP64.  Uses the library's
 * inference work space: calls on one context must not overlap.  Needs the
 * network (MFMG_ERR_UNSUPPORTED otherwise). */
int mfmg_net_infer(mfmg_ctx ctx, int dtype, void* y, const void* b, void* stream);
/* Coarse solver of the V-cycle: MFMG_COARSE_EXACT, _LEARNED (with residual check and
 * fallback, threshold tau) or _ZERO (no coarse correction; for comparison). */
int mfmg_net_mode(mfmg_ctx ctx, int mode, double tau);
/* Number of learned predictions accepted / rejected since the last call and
 * the mean relative residual ||b0 - A0 y|| / ||b0|| of the predictions y
 * (1 for no coarse correction, 0 for the exact solve); resets the counters.
 * Synchronous.  Outputs may be NULL. */
int mfmg_net_counts(mfmg_ctx ctx, int* accepted, int* rejected, double* mean_rel_residual);

/* ---- teardown ------------------------------------------------------------ */
void mfmg_destroy_ctx(mfmg_ctx ctx);
void mfmg_destroy_mesh(mfmg_mesh mesh);
const char* mfmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MFMG_H */
