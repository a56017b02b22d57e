// Host-callable launchers of the device kernels (one HIP translation unit).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mfmg {

// Per-cell record of the operator (one 64-byte line): local entity starts of
// the 27 slots in the batch's LDS vector (0xffff: Dirichlet) and the mask.
struct alignas(64) CellMeta {
  uint16_t loc[28];
  uint32_t mask;
  uint32_t pad;
};
static_assert(sizeof(CellMeta) == 64, "CellMeta must be one 64-byte line");

// Per-level device view of the cell data.
struct CellView {
  const int32_t* ent = nullptr;  // [27][n_cells]
  const uint32_t* mask = nullptr;
  const int32_t* ijk = nullptr;  // [n_cells][3] cell coordinates on its level
  int64_t n_cells = 0;
  int64_t n_dofs = 0;
  int64_t n_shared = 0;
  int k = 1;
  double h0 = 1.0;  // coarse-grid cell size
  double lo = 0.0;  // domain lower corner
  // cell batches of the operator (see dofs.hpp)
  int64_t n_batches = 0;
  const CellMeta* meta = nullptr;     // [n_cells]
  const int32_t* batch_cell = nullptr;
  const int32_t* batch_sh = nullptr;
  const int32_t* batch_ex = nullptr;
  const int32_t* sh_idx = nullptr;
  const int32_t* red_idx = nullptr;
  const int32_t* red_off = nullptr;
  void* partial = nullptr;            // scratch: partial sums, (sh_idx size) x max_rhs x 8 bytes
  // mapped cells (geometry.hpp): coarse-cell map coefficients in FP64 and
  // FP32 ([n0^3][24]), NULL for axis-aligned cubes; n0 coarse cells per axis
  const void* geo64 = nullptr;
  const void* geo32 = nullptr;
  int geo_n0 = 0;
  // deterministic mode: the operator adds its cells' contributions in cell
  // order; the diagonal and the load vector run colour by colour (no two
  // cells of a colour share an entity, plain adds).  color_cells (device)
  // lists the cells colour by colour, color_off (host, n_colors + 1) the
  // colour ranges.
  bool deterministic = false;
  const int32_t* color_cells = nullptr;
  const int64_t* color_off = nullptr;
  int n_colors = 0;
};

// An elementwise step fused into the operator's output: for every DoF i and
// vector v, with t = (A x)_i: none (dst = t), Chebyshev (Saad, Alg. 12.1:
// d = c_dd d + c_r D^{-1} (b - t), x += d; x is the operator's input, updated
// in place once no batch reads it any more) or residual (r = b - t).  b, x,
// d and r are in the storage type, dinv in the arithmetic type.
enum { FUSE_NONE = 0, FUSE_CHEB = 1, FUSE_RESIDUAL = 2 };
struct FusedStep {
  int kind = FUSE_NONE;
  const void* b = nullptr;
  const void* dinv = nullptr;
  void* d = nullptr;
  void* x = nullptr;
  void* r = nullptr;
  double c_dd = 0.0, c_r = 0.0;
};

struct TransferView {
  bool polynomial = false;
  const int32_t* ident_coarse = nullptr;
  const int32_t* ident_fine = nullptr;
  int64_t n_ident = 0;
  const int32_t* refined_coarse = nullptr;
  const int32_t* refined_fine = nullptr;  // [8][n_refined]
  int64_t n_refined = 0;
  const uint8_t* valence = nullptr;       // [27][n_fine_cells]
  // deterministic mode: the restriction runs the groups colour by colour (no
  // two groups of a colour share a coarse entity, plain adds); the group
  // lists are in colour order and ident_off / refined_off (host, colours + 1)
  // give the ranges
  bool deterministic = false;
  const int64_t* ident_off = nullptr;
  int n_ident_colors = 0;
  const int64_t* refined_off = nullptr;
  int n_refined_colors = 0;
};

// dtype: MFMG_F64 / MFMG_F32 / MFMG_BF16 for the vectors named "S"; the
// "acc" vectors are double for F64 and float otherwise.

// dst_acc = A src (every entry written; no initialisation needed)
void launch_vmult(const CellView& c, int dtype, int nv, void* dst_acc, const void* src, hipStream_t s);
// operator application with a fused elementwise step on its output (dst_acc
// unused unless f.kind is FUSE_NONE)
void launch_vmult_fused(const CellView& c, int dtype, int nv, void* dst_acc, const void* src, const FusedStep& f,
                        hipStream_t s);
// Cellwise-constant coefficient on the levels (Section 3.5, interpolate_to_mg
// for a cell field): flag[0] = 1 if a value of c[0..n) is outside
// [1e-30, 1e30] or NaN (flag not cleared here)
void launch_coef_check(int64_t n, const double* c, int* flag, hipStream_t s);
// coarse-level cell values from the next finer level's: a coarse cell that
// is also a fine cell takes its value, a refined one the mean of its eight
// children (summed in child order, x fastest)
void launch_coef_restrict(const TransferView& t, const double* c_fine, double* c_coarse, hipStream_t s);
// write c (rounded to bfloat16) into the coefficient bits of the cell masks
// and of the cells' operator records
void launch_coef_apply(int64_t n_cells, const double* c, uint32_t* mask, CellMeta* meta, hipStream_t s);
// diag (FP64) = diagonal of A
void launch_diagonal(const CellView& c, double* diag, hipStream_t s);
// b (FP64) += load vector; kind 0 const, 1 gaussians (params on device, n_terms per vector)
void launch_rhs(const CellView& c, int kind, const double* dparams, int n_terms, int nv, double* b,
                hipStream_t s);
// dst_fine (S) += P src_coarse (S)
void launch_prolongate(const CellView& fine, const CellView& coarse, const TransferView& t, int dtype, int nv,
                       void* dst_fine, const void* src_coarse, hipStream_t s);
// dst_coarse (S) += P^T src_fine (S)
void launch_restrict(const CellView& fine, const CellView& coarse, const TransferView& t, int dtype, int nv,
                     void* dst_coarse, const void* src_fine, hipStream_t s);

// out[c][n^3] = node values of cell c (constraints applied) for x (FP64)
void launch_distribute(const CellView& c, const double* x, double* out, hipStream_t s);

// ---- vector kernels (n = number of entries, i.e. n_dofs * nv) --------------
void launch_fill(int dtype_bytes, void* x, int64_t n_bytes, hipStream_t s);
// Chebyshev step: first (x = 0): d = dinv*b/theta, x = d;
// else d = c_dd*d + c_r*dinv*(b - t), x += d.   t, dinv: acc type.
void launch_cheb_step(int dtype, int64_t n_dofs, int nv, bool first, double c_dd, double c_r,
                      const void* t, const void* b, const void* dinv, void* d, void* x, hipStream_t s);
// r = b - t (r, b: S; t: acc)
void launch_residual_update(int dtype, int64_t n, const void* b, const void* t, void* r, hipStream_t s);
// cast between FP64 and S
void launch_cast_from_f64(int dtype, int64_t n, const double* src, void* dst, hipStream_t s);
void launch_cast_to_f64(int dtype, int64_t n, const void* src, double* dst, hipStream_t s);
// dst (dtype_dst) = src (dtype_src)
void launch_cast(int dtype_src, int dtype_dst, int64_t n, const void* src, void* dst, hipStream_t s);
// acc -> S
void launch_acc_to_storage(int dtype, int64_t n, const void* acc, void* dst, hipStream_t s);
// dst[dst_idx[q]] = src[src_idx[q]] for q < n, n_vec interleaved values, with a cast
void launch_copy_map(int dtype_src, int dtype_dst, int64_t n, int nv, const int32_t* src_idx, const int32_t* dst_idx,
                     const void* src, void* dst, hipStream_t s);
// a64[idx[q]] = a32[idx[q]] = 0 for q < n
void launch_zero_entries(int64_t n, const int32_t* idx, double* a64, float* a32, hipStream_t s);
// dinv = 1/diag in acc type (0 where diag == 0)
void launch_inverse_diag(int dtype, int64_t n, const double* diag, void* dinv, hipStream_t s);
// x (S) = Ainv (acc type, n0 x n0 row-major) b (S); nv interleaved vectors
void launch_dense_matvec(int dtype, int64_t n0, int nv, const void* Ainv, const void* b, void* x,
                         void* acc_tmp, hipStream_t s);

// ---- FP64 CG helpers --------------------------------------------------------
// partial[blk*nv+v] = sum_i a[i*nv+v]*b[i*nv+v]; result[v] via second stage.
void launch_dot(int64_t n_dofs, int nv, const double* a, const double* b, double* partial, double* result,
                hipStream_t s);
int dot_partials_needed();
// x += alpha[v] p; r -= alpha[v] q   with alpha = num[v]/den[v]
void launch_cg_update_xr(int64_t n_dofs, int nv, const double* num, const double* den, const double* p,
                         const double* q, double* x, double* r, hipStream_t s);
// p = z + beta[v] p  with beta = (num[v] - sub[v]) / den[v] (sub may be null)
void launch_cg_update_p(int64_t n_dofs, int nv, const double* num, const double* sub, const double* den,
                        const double* z, double* p, hipStream_t s);

}  // namespace mfmg
