// Level set-up and the multigrid algorithms on top of the kernels:
// Chebyshev-Jacobi smoothing (Section 3.3), the V-cycle (Algorithms 1-2,
// global-coarsening branch), the exact coarse solver and PCG (Section 2).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <thread>
#include <unordered_map>

#include "context.hpp"
#include "fe1d.hpp"
#include "net.hpp"

namespace mfmg {

namespace {

int acc_dtype(int dtype) { return dtype == MFMG_F64 ? MFMG_F64 : MFMG_F32; }

void sync(hipStream_t s) { MFMG_HIP(hipStreamSynchronize(s)); }

// Largest eigenvalue of a small symmetric matrix (cyclic Jacobi rotations).
double max_eig_sym(std::vector<double> A, int n) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < n; ++r) {
          double arp = A[r * n + p], arq = A[r * n + q];
          A[r * n + p] = c * arp - s * arq;
          A[r * n + q] = s * arp + c * arq;
        }
        for (int r = 0; r < n; ++r) {
          double apr = A[p * n + r], aqr = A[q * n + r];
          A[p * n + r] = c * apr - s * aqr;
          A[q * n + r] = s * apr + c * aqr;
        }
      }
  }
  double m = -1e300;
  for (int i = 0; i < n; ++i) m = std::max(m, A[i * n + i]);
  return m;
}

// Dense inverse of an SPD matrix: Cholesky A = L L^T, then columns of A^{-1}
// by forward/backward substitution (columns in parallel threads).
std::vector<double> spd_inverse(std::vector<double> A, int64_t n) {
  for (int64_t j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int64_t q = 0; q < j; ++q) d -= A[j * n + q] * A[j * n + q];
    MFMG_REQUIRE(d > 0.0, MFMG_ERR_BREAKDOWN, "coarse matrix is not positive definite");
    d = std::sqrt(d);
    A[j * n + j] = d;
    const double inv = 1.0 / d;
    const int64_t rows = n - j - 1;
    auto work = [&](int64_t r0, int64_t r1) {
      for (int64_t i = r0; i < r1; ++i) {
        double s = A[i * n + j];
        const double* ai = &A[i * n];
        const double* aj = &A[j * n];
        for (int64_t q = 0; q < j; ++q) s -= ai[q] * aj[q];
        A[i * n + j] = s * inv;
      }
    };
    if (rows > 256) {
      unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
      std::vector<std::thread> th;
      for (unsigned t = 0; t < nt; ++t) {
        int64_t r0 = j + 1 + rows * t / nt, r1 = j + 1 + rows * (t + 1) / nt;
        th.emplace_back(work, r0, r1);
      }
      for (auto& x : th) x.join();
    } else {
      work(j + 1, n);
    }
  }
  std::vector<double> inv(static_cast<size_t>(n * n), 0.0);
  auto cols = [&](int64_t c0, int64_t c1) {
    std::vector<double> y(n);
    for (int64_t c = c0; c < c1; ++c) {
      for (int64_t i = 0; i < n; ++i) {
        double s = (i == c) ? 1.0 : 0.0;
        for (int64_t q = 0; q < i; ++q) s -= A[i * n + q] * y[q];
        y[i] = s / A[i * n + i];
      }
      for (int64_t i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int64_t q = i + 1; q < n; ++q) s -= A[q * n + i] * inv[q * n + c];
        inv[i * n + c] = s / A[i * n + i];
      }
    }
  };
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 256) nt = 1;
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) th.emplace_back(cols, n * t / nt, n * (t + 1) / nt);
  for (auto& x : th) x.join();
  return inv;
}

std::vector<std::pair<int, int>> level_pairs(int n_meshes, int k, int scheme) {
  // (mesh index, degree), coarse to fine; mesh index 0 = coarse grid
  std::vector<int> degs{k};
  while (degs.back() > 1) degs.push_back(degs.back() / 2);  // fine to coarse
  std::vector<std::pair<int, int>> p;                       // fine to coarse
  const int fine = n_meshes - 1;
  if (scheme == MFMG_SCHEME_H) {
    for (int m = fine; m >= 0; --m) p.push_back({m, k});
  } else if (scheme == MFMG_SCHEME_P_THEN_H) {
    for (int d : degs) p.push_back({fine, d});
    for (int m = fine - 1; m >= 0; --m) p.push_back({m, 1});
  } else if (scheme == MFMG_SCHEME_H_THEN_P) {
    for (int m = fine; m >= 0; --m) p.push_back({m, k});
    for (size_t i = 1; i < degs.size(); ++i) p.push_back({0, degs[i]});
  } else if (scheme == MFMG_SCHEME_HP) {
    // mesh and degree coarsened together while both can be; then whichever is left
    size_t d = 0;
    int m = fine;
    p.push_back({m, degs[0]});
    while (m > 0 || d + 1 < degs.size()) {
      if (m > 0) --m;
      if (d + 1 < degs.size()) ++d;
      p.push_back({m, degs[d]});
    }
  } else {
    throw Error(MFMG_ERR_INVALID_ARG, "unknown level scheme");
  }
  std::reverse(p.begin(), p.end());
  return p;
}

void estimate_eigenvalues(Context& ctx, Level& L, int iters, double safety, double range, hipStream_t s) {
  const int64_t n = L.n_dofs;
  if (n == 0) { L.lmin = 1.0 / range; L.lmax = 1.0; return; }
  DeviceArray<double> x(n), r(n), z(n), p(n), q(n), part(dot_partials_needed()), sc(4);
  std::vector<double> ones(n, 1.0);
  MFMG_HIP(hipMemcpy(r.ptr, ones.data(), n * 8, hipMemcpyHostToDevice));
  const double* dinv = reinterpret_cast<const double*>(L.dinv.ptr);
  std::vector<double> hd(n);
  // z = D^{-1} r on the host-visible path: reuse the Chebyshev kernel with b=r
  auto precond = [&](double* dst, const double* src) {
    launch_cheb_step(MFMG_F64, n, 1, true, 0.0, 1.0, nullptr, src, dinv, dst, x.ptr, s);
  };
  precond(z.ptr, r.ptr);
  MFMG_HIP(hipMemcpyAsync(p.ptr, z.ptr, n * 8, hipMemcpyDeviceToDevice, s));
  launch_dot(n, 1, r.ptr, z.ptr, part.ptr, sc.ptr + 0, s);  // rz
  double rz;
  MFMG_HIP(hipMemcpyAsync(&rz, sc.ptr, 8, hipMemcpyDeviceToHost, s));
  sync(s);
  std::vector<double> alphas, betas;
  for (int it = 0; it < std::min<int64_t>(iters, n); ++it) {
    launch_vmult(L.view, MFMG_F64, 1, q.ptr, p.ptr, s);
    launch_dot(n, 1, p.ptr, q.ptr, part.ptr, sc.ptr + 1, s);  // pAp
    double pap;
    MFMG_HIP(hipMemcpyAsync(&pap, sc.ptr + 1, 8, hipMemcpyDeviceToHost, s));
    sync(s);
    if (!(pap > 0.0) || !(rz > 0.0)) break;
    // r -= alpha q (x unused)
    launch_cg_update_xr(n, 1, sc.ptr + 0, sc.ptr + 1, p.ptr, q.ptr, x.ptr, r.ptr, s);
    precond(z.ptr, r.ptr);
    launch_dot(n, 1, r.ptr, z.ptr, part.ptr, sc.ptr + 2, s);  // rz_new
    double rzn;
    MFMG_HIP(hipMemcpyAsync(&rzn, sc.ptr + 2, 8, hipMemcpyDeviceToHost, s));
    sync(s);
    const double alpha = rz / pap, beta = rzn / rz;
    alphas.push_back(alpha);
    betas.push_back(beta);
    if (!(rzn > 0.0)) break;
    launch_cg_update_p(n, 1, sc.ptr + 2, nullptr, sc.ptr + 0, z.ptr, p.ptr, s);
    MFMG_HIP(hipMemcpyAsync(sc.ptr, sc.ptr + 2, 8, hipMemcpyDeviceToDevice, s));
    rz = rzn;
  }
  const int m = static_cast<int>(alphas.size());
  double lam = 1.0;
  if (m > 0) {
    std::vector<double> T(m * m, 0.0);
    for (int j = 0; j < m; ++j) {
      T[j * m + j] = 1.0 / alphas[j] + (j > 0 ? betas[j - 1] / alphas[j - 1] : 0.0);
      if (j + 1 < m) T[j * m + j + 1] = T[(j + 1) * m + j] = std::sqrt(betas[j]) / alphas[j];
    }
    lam = max_eig_sym(T, m);
  }
  L.lmax = safety * lam;
  L.lmin = L.lmax / range;
}

template <typename T>
void upload_into(DeviceArray<T>& d, const std::vector<T>& h) { d.upload(h); }

}  // namespace

namespace {
// Device data of one level from its host description; `work` allocates the
// V-cycle work vectors.
void init_level(Context& ctx, Level& L, const LevelDofs& H, double lo, bool work, hipStream_t s) {
  L.n_dofs = H.n_dofs;
  L.n_cells = H.n_cells;
  L.n_hanging = H.n_hanging_cells;
  L.ent.upload(H.ent);
  L.mask.upload(H.mask);
  std::vector<int32_t> ijk(3 * H.n_cells);
  for (int64_t c = 0; c < H.n_cells; ++c) {
    ijk[3 * c] = static_cast<int32_t>(H.cells[c].i);
    ijk[3 * c + 1] = static_cast<int32_t>(H.cells[c].j);
    ijk[3 * c + 2] = static_cast<int32_t>(H.cells[c].k);
  }
  L.ijk.upload(ijk);
  L.host_ijk = ijk;
  L.host_levels.resize(H.n_cells);
  for (int64_t c = 0; c < H.n_cells; ++c) L.host_levels[c] = H.cells[c].level;
  L.view.ent = L.ent.ptr;
  L.view.mask = L.mask.ptr;
  L.view.ijk = L.ijk.ptr;
  L.view.n_cells = H.n_cells;
  L.view.n_dofs = H.n_dofs;
  L.view.n_shared = H.n_shared;
  L.view.k = L.k;
  L.view.h0 = H.h0;
  L.view.lo = lo;
  {
    std::vector<CellMeta> meta(H.n_cells);
    for (int64_t c = 0; c < H.n_cells; ++c) {
      for (int sl = 0; sl < N_SLOTS; ++sl) meta[c].loc[sl] = H.loc[sl * H.n_cells + c];
      meta[c].loc[27] = 0xffff;
      meta[c].mask = H.mask[c];
      meta[c].pad = 0;
    }
    L.meta.upload(meta);
  }
  L.batch_cell.upload(H.batch_cell_off);
  L.batch_sh.upload(H.batch_sh_off);
  L.batch_ex.upload(H.batch_ex_off);
  L.sh_idx.upload(H.sh_idx);
  L.red_idx.upload(H.red_idx);
  L.red_off.upload(H.red_off);
  L.partial.alloc(std::max<size_t>(1, H.sh_idx.size()) * ctx.max_rhs * 8);
  L.view.n_batches = H.n_batches;
  L.view.meta = L.meta.ptr;
  L.view.batch_cell = L.batch_cell.ptr;
  L.view.batch_sh = L.batch_sh.ptr;
  L.view.batch_ex = L.batch_ex.ptr;
  L.view.sh_idx = L.sh_idx.ptr;
  L.view.red_idx = L.red_idx.ptr;
  L.view.red_off = L.red_off.ptr;
  L.view.partial = L.partial.ptr;
  if (ctx.geo.kind != 0) {
    L.view.geo64 = ctx.geo64.ptr;
    L.view.geo32 = ctx.geo32.ptr;
    L.view.geo_n0 = ctx.geo_n0;
  }
  const int64_t nrhs = L.n_dofs * ctx.max_rhs;
  const size_t sb = dtype_size(L.dtype);
  if (work) {
    L.x.alloc(nrhs * sb);
    L.b.alloc(nrhs * sb);
    L.r.alloc(nrhs * sb);
    L.d.alloc(nrhs * 8);
    L.tmp_cast.alloc(nrhs * 8);
  }
  L.t.alloc(nrhs * 8);
  if (ctx.desc.deterministic) {
    std::vector<int32_t> cells;
    colour_cells(H, cells, L.color_off);
    L.color_cells.upload(cells);
    L.view.deterministic = true;
    L.view.color_cells = L.color_cells.ptr;
    L.view.color_off = L.color_off.data();
    L.view.n_colors = static_cast<int>(L.color_off.size()) - 1;
  }
  L.diag.alloc(L.n_dofs);
  L.dinv.alloc(L.n_dofs * 8 * 2);  // double copy, then float copy
  launch_diagonal(L.view, L.diag.ptr, s);
  launch_inverse_diag(MFMG_F64, L.n_dofs, L.diag.ptr, L.dinv.ptr, s);
  launch_inverse_diag(MFMG_F32, L.n_dofs, L.diag.ptr, L.dinv.ptr + L.n_dofs * 8, s);
}

void init_transfer(Level& L, const TransferDofs& T, bool poly) {
  L.has_transfer = true;
  if (!T.ident_off.empty() || !T.refined_off.empty()) {  // coloured groups (deterministic mode)
    L.tr_ident_off = T.ident_off;
    L.tr_refined_off = T.refined_off;
    L.tview.deterministic = true;
    L.tview.ident_off = L.tr_ident_off.data();
    L.tview.n_ident_colors = static_cast<int>(L.tr_ident_off.size()) - 1;
    L.tview.refined_off = L.tr_refined_off.data();
    L.tview.n_refined_colors = static_cast<int>(L.tr_refined_off.size()) - 1;
  }
  L.tr_ident_c.upload(T.ident_coarse);
  L.tr_ident_f.upload(T.ident_fine);
  L.tr_ref_c.upload(T.refined_coarse);
  L.tr_ref_f.upload(T.refined_fine);
  L.tr_valence.upload(T.valence);
  L.tview.polynomial = poly;
  L.tview.ident_coarse = L.tr_ident_c.ptr;
  L.tview.ident_fine = L.tr_ident_f.ptr;
  L.tview.n_ident = static_cast<int64_t>(T.ident_coarse.size());
  L.tview.refined_coarse = L.tr_ref_c.ptr;
  L.tview.refined_fine = L.tr_ref_f.ptr;
  L.tview.n_refined = static_cast<int64_t>(T.refined_coarse.size());
  L.tview.valence = L.tr_valence.ptr;
}

int level_dtype(const mfmg_level_desc& desc, int l) {
  const int dt = desc.n_level_dtype <= 0 ? MFMG_F64 : desc.level_dtype[std::min(l, desc.n_level_dtype - 1)];
  MFMG_REQUIRE(dt >= MFMG_F64 && dt <= MFMG_BF16, MFMG_ERR_UNSUPPORTED, "level dtype");
  return dt;
}

// Local smoothing (Section 2.1): one level per refinement level, holding all
// of its cells; refinement-edge DoFs get a zero inverse diagonal, so that the
// Chebyshev smoother acts on A_SS and keeps the edge values.  The copy maps
// of Algorithm 1 pair the entities of the leaves of each level (interior
// ones only) with the same entities of the active mesh.
void setup_local_smoothing(Context& ctx, const mfmg_level_desc& desc, std::vector<LevelDofs>& host, hipStream_t s) {
  MFMG_REQUIRE(desc.dirichlet != 0, MFMG_ERR_UNSUPPORTED, "local smoothing needs Dirichlet boundary conditions");
  MFMG_REQUIRE(desc.drop_coarse == 0, MFMG_ERR_UNSUPPORTED,
               "local smoothing switches to the coarse solver only on a level that covers the domain");
  const Octree& tree = ctx.meshes.back();
  std::vector<int> lv;
  for (int l = 0; l <= tree.n_levels(); ++l)
    if (l == 0 || (l - 1 < tree.n_levels() && !tree.refined[l - 1].empty())) lv.push_back(l);
  // LS_THEN_P: polynomial levels on the coarse grid below it (degrees 1, 2,
  // ..., floor(k/2); Section 2.3), without edge or copied right-hand side
  std::vector<int> pdeg;
  if (desc.scheme == MFMG_SCHEME_LS_THEN_P)
    for (int d = desc.degree / 2; d >= 1; d /= 2) pdeg.insert(pdeg.begin(), d);
  const int np = static_cast<int>(pdeg.size());
  MFMG_REQUIRE(lv.size() + np <= MFMG_MAX_LEVELS, MFMG_ERR_UNSUPPORTED, "too many levels");
  const int nl = static_cast<int>(lv.size()) + np;
  ctx.ls = true;
  ctx.levels.clear();
  ctx.levels.resize(nl);
  host.assign(nl, LevelDofs());
  for (int l = 0; l < nl; ++l) {
    Level& L = ctx.levels[l];
    const bool poly_level = l < np;
    L.mesh = poly_level ? 0 : static_cast<int>(ctx.meshes.size()) - 1;
    L.only_level = poly_level ? -1 : lv[l - np];
    L.k = poly_level ? pdeg[l] : desc.degree;
    L.dtype = level_dtype(desc, l);
    MFMG_REQUIRE(L.dtype == ctx.levels[0].dtype, MFMG_ERR_UNSUPPORTED,
                 "local smoothing needs one storage type on all levels");
    host[l] = poly_level ? build_level_dofs(ctx.meshes[0], L.k, true, false, -1, &ctx.coef, &tree)
                         : build_level_dofs(tree, L.k, true, false, L.only_level, &ctx.coef, &tree);
    MFMG_REQUIRE(l > np || host[l].n_edge_dofs == 0, MFMG_ERR_INVALID_ARG, "the coarse grid has an edge");
    init_level(ctx, L, host[l], tree.lo, true, s);
    L.n_edge = host[l].n_edge_dofs;
    L.host_edge = host[l].dof_edge;
    std::vector<int32_t> edge;
    edge.reserve(L.n_edge);
    for (size_t i = 0; i < host[l].dof_edge.size(); ++i)
      if (host[l].dof_edge[i]) edge.push_back(static_cast<int32_t>(i));
    L.edge_idx.upload(edge);
    launch_zero_entries(L.n_edge, L.edge_idx.ptr, reinterpret_cast<double*>(L.dinv.ptr),
                        reinterpret_cast<float*>(L.dinv.ptr + L.n_dofs * 8), s);
  }
  for (int l = 1; l < nl; ++l) {
    const bool poly = ctx.levels[l - 1].k != ctx.levels[l].k;
    init_transfer(ctx.levels[l], build_transfer(host[l], host[l - 1], poly, !poly, ctx.desc.deterministic != 0),
                  poly);
  }
  // the active mesh (the outer solver's operator), FP64
  LevelDofs A = build_level_dofs(tree, desc.degree, true, false, -1, &ctx.coef);
  Level& F = ctx.active;
  F.mesh = static_cast<int>(ctx.meshes.size()) - 1;
  F.k = desc.degree;
  F.dtype = MFMG_F64;
  init_level(ctx, F, A, tree.lo, false, s);
  // copy maps; every active DoF belongs to exactly one level
  const EntityIndex index(A);
  std::vector<uint8_t> covered(A.n_dofs, 0);
  for (int l = np; l < nl; ++l) {
    std::vector<int32_t> cl, ca;
    ls_copy_pairs(host[l], A, index, cl, ca);
    for (int32_t a : ca) {
      MFMG_REQUIRE(!covered[a], MFMG_ERR_INVALID_ARG, "copy map: active DoF on two levels");
      covered[a] = 1;
    }
    Level& L = ctx.levels[l];
    L.n_copy = static_cast<int64_t>(cl.size());
    L.cp_level.upload(cl);
    L.cp_active.upload(ca);
  }
  for (int64_t i = 0; i < A.n_dofs; ++i)
    MFMG_REQUIRE(covered[i], MFMG_ERR_INVALID_ARG, "copy map: active DoF on no level");
}
}  // namespace

namespace {
// dense A^(0) of the coarse level (from its host description) and its inverse
void setup_coarse_solver(Context& ctx) {
  const LevelDofs& H = ctx.coarse_host;
  std::vector<double> A = assemble_dense(H, Tables1D(H.k), ctx.geo.kind ? &ctx.geo_host : nullptr, ctx.geo_n0);
  ctx.coarse_A64.upload(A);
  std::vector<double> inv = spd_inverse(std::move(A), ctx.n0);
  std::vector<float> inv32(inv.begin(), inv.end());
  ctx.coarse_inv64.upload(inv);
  ctx.coarse_inv32.upload(inv32);
}
}  // namespace

void setup_context(Context& ctx, const mfmg_mesh_s& mesh, const mfmg_level_desc& desc, hipStream_t s) {
  MFMG_REQUIRE(desc.degree >= 1 && desc.degree <= 6, MFMG_ERR_UNSUPPORTED, "degree must be in [1, 6]");
  ctx.desc = desc;
  ctx.coef.kind = desc.coef_kind;
  for (int i = 0; i < 8; ++i) ctx.coef.p[i] = desc.coef_params[i];
  MFMG_REQUIRE(desc.coef_kind >= 0 && desc.coef_kind <= 2, MFMG_ERR_INVALID_ARG, "unknown coefficient kind");
  MFMG_REQUIRE(!desc.fmg_start || (desc.scheme != MFMG_SCHEME_LS && desc.scheme != MFMG_SCHEME_LS_THEN_P),
               MFMG_ERR_UNSUPPORTED, "full multigrid runs on global-coarsening levels");
  ctx.stream = s;
  ctx.meshes = mesh.gc;
  ctx.geo.kind = desc.geom_kind;
  for (int i = 0; i < 8; ++i) ctx.geo.p[i] = desc.geom_params[i];
  MFMG_REQUIRE(desc.geom_kind >= 0 && desc.geom_kind <= 2, MFMG_ERR_INVALID_ARG, "unknown geometry kind");
  if (ctx.geo.kind != 0) {
    MFMG_REQUIRE(desc.scheme != MFMG_SCHEME_LS && desc.scheme != MFMG_SCHEME_LS_THEN_P, MFMG_ERR_UNSUPPORTED,
                 "mapped cells are built for global-coarsening levels");
    const Octree& g0 = ctx.meshes[0];
    ctx.geo_n0 = g0.n0;
    ctx.geo_host = geometry_table(ctx.geo, g0.n0, g0.lo, g0.hi);
    // every coarse-cell map must keep its orientation (det J > 0 at the
    // corners and the centre of each coarse cell)
    for (size_t c = 0; c * 24 < ctx.geo_host.size(); ++c)
      for (int q = 0; q < 9; ++q) {
        const double t1 = q < 8 ? (q & 1) : 0.5, t2 = q < 8 ? ((q >> 1) & 1) : 0.5, t3 = q < 8 ? ((q >> 2) & 1) : 0.5;
        double J[3][3];
        geo_jacobian<double>(&ctx.geo_host[c * 24], t1, t2, t3, J);
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        MFMG_REQUIRE(det > 0.0, MFMG_ERR_INVALID_ARG, "geometry: a coarse cell map is not orientation preserving");
      }
    ctx.geo64.upload(ctx.geo_host);
    std::vector<float> g32(ctx.geo_host.begin(), ctx.geo_host.end());
    ctx.geo32.upload(g32);
  }
  ctx.max_rhs = desc.max_rhs > 0 ? desc.max_rhs : 1;
  MFMG_REQUIRE(ctx.max_rhs <= 8, MFMG_ERR_UNSUPPORTED, "max_rhs must be <= 8");
  ctx.cheb_degree = desc.cheb_degree > 0 ? desc.cheb_degree : 3;
  const double range = desc.smoothing_range > 0 ? desc.smoothing_range : 20.0;
  const double safety = desc.eig_safety > 0 ? desc.eig_safety : 1.2;
  const int eig_it = desc.eig_iterations > 0 ? desc.eig_iterations : 15;
  std::vector<LevelDofs> host;
  if (desc.scheme == MFMG_SCHEME_LS || desc.scheme == MFMG_SCHEME_LS_THEN_P) {
    setup_local_smoothing(ctx, desc, host, s);
  } else {
    auto pairs = level_pairs(static_cast<int>(ctx.meshes.size()), desc.degree, desc.scheme);
    MFMG_REQUIRE(desc.drop_coarse >= 0 && desc.drop_coarse < static_cast<int>(pairs.size()), MFMG_ERR_INVALID_ARG,
                 "drop_coarse must leave at least one level");
    pairs.erase(pairs.begin(), pairs.begin() + desc.drop_coarse);  // early switch to the coarse solver
    MFMG_REQUIRE(pairs.size() <= MFMG_MAX_LEVELS, MFMG_ERR_UNSUPPORTED, "too many levels");
    const int nl = static_cast<int>(pairs.size());
    ctx.levels.clear();
    ctx.levels.resize(nl);
    host.resize(nl);
    for (int l = 0; l < nl; ++l) {
      Level& L = ctx.levels[l];
      L.mesh = pairs[l].first;
      L.k = pairs[l].second;
      L.dtype = level_dtype(desc, l);
      host[l] = build_level_dofs(ctx.meshes[L.mesh], L.k, desc.dirichlet != 0, false, -1, &ctx.coef,
                                 &ctx.meshes.back());
      init_level(ctx, L, host[l], ctx.meshes[L.mesh].lo, true, s);
    }
    for (int l = 1; l < nl; ++l) {
      const bool poly = ctx.levels[l - 1].mesh == ctx.levels[l].mesh;
      init_transfer(ctx.levels[l], build_transfer(host[l], host[l - 1], poly, false, ctx.desc.deterministic != 0),
                    poly);
    }
  }
  const int nl = static_cast<int>(ctx.levels.size());
  sync(s);
  for (int l = 1; l < nl; ++l) estimate_eigenvalues(ctx, ctx.levels[l], eig_it, safety, range, s);
  // exact coarse solver
  ctx.n0 = ctx.levels[0].n_dofs;
  if (desc.dirichlet) {  // (the pure Neumann coarse matrix is singular)
    MFMG_REQUIRE(ctx.n0 <= 12000, MFMG_ERR_UNSUPPORTED, "coarse level too large for the dense direct solver");
    ctx.coarse_host = host[0];
    setup_coarse_solver(ctx);
  }
  // learned coarse correction (available for small coarse levels without hanging nodes)
  if (desc.dirichlet && ctx.n0 > 0 && ctx.n0 <= 2048 && host[0].n_hanging_cells == 0 && net_supported(host[0].k))
    net_setup(ctx, host[0]);
  // PCG work space
  const int64_t nf = ctx.fine().n_dofs * ctx.max_rhs;
  ctx.cg_r.alloc(nf);
  ctx.cg_p.alloc(nf);
  ctx.cg_q.alloc(nf);
  ctx.cg_z.alloc(nf);
  ctx.cg_zold.alloc(nf);
  ctx.cg_partial.alloc(static_cast<size_t>(dot_partials_needed()) * 8);
  ctx.cg_scalar.alloc(8 * 8);
  ctx.host_scalar.assign(8 * 8, 0.0);
  ctx.rhs_params.alloc(static_cast<size_t>(5) * 8 * ctx.max_rhs);  // 8 Gaussians per vector
  sync(s);
}

// ---------------------------------------------------------------------------
void level_vmult(Context& ctx, int l, int dtype, int nv, void* dst_acc, const void* src, hipStream_t s) {
  Level& L = ctx.level(l);
  launch_vmult(L.view, dtype, nv, dst_acc, src, s);
}

void level_smooth(Context& ctx, int l, int nv, void* x, const void* b, bool x_is_zero, double lmin, double lmax,
                  hipStream_t s) {
  Level& L = ctx.level(l);
  const int dt = L.dtype;
  const void* dinv = acc_dtype(dt) == MFMG_F64 ? static_cast<const void*>(L.dinv.ptr)
                                               : static_cast<const void*>(L.dinv.ptr + L.n_dofs * 8);
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  // each operator application on one vector carries the Chebyshev update of
  // its output (exclusive DoFs in the batch kernel, shared DoFs in the pass
  // after it); several interleaved vectors are updated by the contiguous
  // vector kernel instead
  if (nv > 1) {
    if (x_is_zero) {
      launch_cheb_step(dt, L.n_dofs, nv, true, 0.0, 1.0 / theta, nullptr, b, dinv, L.d.ptr, x, s);
    } else {
      launch_vmult(L.view, dt, nv, L.t.ptr, x, s);
      launch_cheb_step(dt, L.n_dofs, nv, false, 0.0, 1.0 / theta, L.t.ptr, b, dinv, L.d.ptr, x, s);
    }
    for (int it = 1; it < ctx.cheb_degree; ++it) {
      const double rho_new = 1.0 / (2.0 * sigma - rho);
      launch_vmult(L.view, dt, nv, L.t.ptr, x, s);
      launch_cheb_step(dt, L.n_dofs, nv, false, rho_new * rho, 2.0 * rho_new / delta, L.t.ptr, b, dinv, L.d.ptr, x,
                       s);
      rho = rho_new;
    }
    return;
  }
  FusedStep f;
  f.kind = FUSE_CHEB;
  f.b = b;
  f.dinv = dinv;
  f.d = L.d.ptr;
  f.x = x;
  if (x_is_zero) {
    launch_cheb_step(dt, L.n_dofs, nv, true, 0.0, 1.0 / theta, nullptr, b, dinv, L.d.ptr, x, s);
  } else {
    f.c_dd = 0.0;
    f.c_r = 1.0 / theta;
    launch_vmult_fused(L.view, dt, nv, nullptr, x, f, s);
  }
  for (int it = 1; it < ctx.cheb_degree; ++it) {
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    f.c_dd = rho_new * rho;
    f.c_r = 2.0 * rho_new / delta;
    launch_vmult_fused(L.view, dt, nv, nullptr, x, f, s);
    rho = rho_new;
  }
}

void level_residual(Context& ctx, int l, int nv, void* r, const void* b, const void* x, hipStream_t s) {
  Level& L = ctx.level(l);
  if (nv > 1) {  // (see level_smooth)
    launch_vmult(L.view, L.dtype, nv, L.t.ptr, x, s);
    launch_residual_update(L.dtype, L.n_dofs * nv, b, L.t.ptr, r, s);
    return;
  }
  FusedStep f;  // r = b - A x on the operator's output
  f.kind = FUSE_RESIDUAL;
  f.b = b;
  f.r = r;
  launch_vmult_fused(L.view, L.dtype, nv, nullptr, x, f, s);
}

void level_prolongate_add(Context& ctx, int fine, int dtype, int nv, void* dst, const void* src, hipStream_t s) {
  MFMG_REQUIRE(fine >= 1 && fine < static_cast<int>(ctx.levels.size()), MFMG_ERR_INVALID_ARG, "fine level");
  Level& F = ctx.levels[fine];
  Level& C = ctx.levels[fine - 1];
  launch_prolongate(F.view, C.view, F.tview, dtype, nv, dst, src, s);
}

void level_restrict_add(Context& ctx, int fine, int dtype, int nv, void* dst, const void* src, hipStream_t s) {
  MFMG_REQUIRE(fine >= 1 && fine < static_cast<int>(ctx.levels.size()), MFMG_ERR_INVALID_ARG, "fine level");
  Level& F = ctx.levels[fine];
  Level& C = ctx.levels[fine - 1];
  launch_restrict(F.view, C.view, F.tview, dtype, nv, dst, src, s);
}

void coarse_solve(Context& ctx, int dtype, int nv, void* x, const void* b, hipStream_t s) {
  const void* inv = dtype == MFMG_F64 ? static_cast<const void*>(ctx.coarse_inv64.ptr)
                                      : static_cast<const void*>(ctx.coarse_inv32.ptr);
  launch_dense_matvec(dtype, ctx.n0, nv, inv, b, x, nullptr, s);
}

namespace {
void coarse_level_solve(Context& ctx, int nv, hipStream_t s);

// C.b = P^T src (src on level l, in its storage type), through a cast when
// the two levels store different types
void restrict_into_zeroed(Context& ctx, int l, int nv, const void* src, hipStream_t s) {
  Level& L = ctx.levels[l];
  Level& C = ctx.levels[l - 1];
  launch_fill(0, C.b.ptr, C.n_dofs * nv * static_cast<int64_t>(dtype_size(C.dtype)), s);
  if (C.dtype == L.dtype) {
    level_restrict_add(ctx, l, L.dtype, nv, C.b.ptr, src, s);
  } else {
    launch_fill(0, C.tmp_cast.ptr, C.n_dofs * nv * static_cast<int64_t>(dtype_size(L.dtype)), s);
    level_restrict_add(ctx, l, L.dtype, nv, C.tmp_cast.ptr, src, s);
    launch_cast(L.dtype, C.dtype, C.n_dofs * nv, C.tmp_cast.ptr, C.b.ptr, s);
  }
}

// L.x += P C.x
void prolongate_from_coarse(Context& ctx, int l, int nv, hipStream_t s) {
  Level& L = ctx.levels[l];
  Level& C = ctx.levels[l - 1];
  if (C.dtype == L.dtype) {
    level_prolongate_add(ctx, l, L.dtype, nv, L.x.ptr, C.x.ptr, s);
  } else {
    launch_cast(C.dtype, L.dtype, C.n_dofs * nv, C.x.ptr, C.tmp_cast.ptr, s);
    level_prolongate_add(ctx, l, L.dtype, nv, L.x.ptr, C.tmp_cast.ptr, s);
  }
}

// Algorithm 2 (global-coarsening branch) on A^(l) x = b^(l); presmoothing
// starts from x = 0 unless `x_zero` is false (then from the given L.x)
void vcycle_level(Context& ctx, int l, int nv, hipStream_t s, bool x_zero = true) {
  Level& L = ctx.levels[l];
  if (l == 0) {
    coarse_level_solve(ctx, nv, s);
    return;
  }
  level_smooth(ctx, l, nv, L.x.ptr, L.b.ptr, x_zero, L.lmin, L.lmax, s);   // presmoothing
  level_residual(ctx, l, nv, L.r.ptr, L.b.ptr, L.x.ptr, s);                // residual
  restrict_into_zeroed(ctx, l, nv, L.r.ptr, s);                           // restriction
  vcycle_level(ctx, l - 1, nv, s);                                         // coarse correction
  prolongate_from_coarse(ctx, l, nv, s);                                   // prolongation
  level_smooth(ctx, l, nv, L.x.ptr, L.b.ptr, false, L.lmin, L.lmax, s);  // postsmoothing
}
}  // namespace

void fmg(Context& ctx, int nv, double* x, const double* b, int cycles, hipStream_t s) {
  MFMG_REQUIRE(!ctx.ls, MFMG_ERR_UNSUPPORTED, "full multigrid runs on global-coarsening levels");
  MFMG_REQUIRE(nv >= 1 && nv <= ctx.max_rhs, MFMG_ERR_INVALID_ARG, "n_vec exceeds max_rhs");
  MFMG_REQUIRE(cycles >= 1 && cycles <= 16, MFMG_ERR_INVALID_ARG, "cycles must be in [1, 16]");
  const int top = static_cast<int>(ctx.levels.size()) - 1;
  Level& F = ctx.levels[top];
  launch_cast(MFMG_F64, F.dtype, F.n_dofs * nv, b, F.b.ptr, s);
  for (int l = top; l >= 1; --l) restrict_into_zeroed(ctx, l, nv, ctx.levels[l].b.ptr, s);  // b^(l-1) = P^T b^(l)
  coarse_level_solve(ctx, nv, s);
  for (int l = 1; l <= top; ++l) {
    Level& L = ctx.levels[l];
    launch_fill(0, L.x.ptr, L.n_dofs * nv * static_cast<int64_t>(dtype_size(L.dtype)), s);
    prolongate_from_coarse(ctx, l, nv, s);  // initial guess from the coarser level
    for (int c = 0; c < cycles; ++c) vcycle_level(ctx, l, nv, s, false);
  }
  launch_cast(F.dtype, MFMG_F64, F.n_dofs * nv, F.x.ptr, x, s);
}

namespace {
void coarse_level_solve(Context& ctx, int nv, hipStream_t s) {
  Level& L = ctx.levels[0];
  NetState& N = ctx.net;
  if (N.rec_count < N.rec_capacity && nv == 1) {
    launch_cast(L.dtype, MFMG_F64, L.n_dofs, L.b.ptr, N.record.ptr + static_cast<int64_t>(N.rec_count) * L.n_dofs, s);
    ++N.rec_count;
  }
  if (N.mode != MFMG_COARSE_EXACT && nv == 1) net_coarse_solve(ctx, L.dtype, L.x.ptr, L.b.ptr, s);
  else coarse_solve(ctx, L.dtype, nv, L.x.ptr, L.b.ptr, s);
}

// Algorithm 2, local-smoothing branch.  The edge DoFs have a zero inverse
// diagonal: presmoothing from x = 0 leaves x_E = 0, so the residual gives
// b_S - A_SS x_S on interior DoFs and -A_ES x_S on edge DoFs (b_E is 0: the
// copy to the levels writes interior DoFs only, and no refined cell of a
// level touches its edge on a one-irregular mesh).  The restriction adds to
// the coarser right-hand side, which already holds that level's share of the
// copied b.  The prolongation also sets x_E; the postsmoother's operator then
// applies A_SS x_S + A_SE x_E while it keeps x_E, which is the edge step
// b_S - A_SE x_E folded into the smoother.
void ls_vcycle_level(Context& ctx, int l, int nv, hipStream_t s) {
  if (l == 0) {
    coarse_level_solve(ctx, nv, s);
    return;
  }
  Level& L = ctx.levels[l];
  Level& C = ctx.levels[l - 1];
  level_smooth(ctx, l, nv, L.x.ptr, L.b.ptr, true, L.lmin, L.lmax, s);
  level_residual(ctx, l, nv, L.r.ptr, L.b.ptr, L.x.ptr, s);
  level_restrict_add(ctx, l, L.dtype, nv, C.b.ptr, L.r.ptr, s);
  ls_vcycle_level(ctx, l - 1, nv, s);
  level_prolongate_add(ctx, l, L.dtype, nv, L.x.ptr, C.x.ptr, s);
  level_smooth(ctx, l, nv, L.x.ptr, L.b.ptr, false, L.lmin, L.lmax, s);
}
}  // namespace

void copy_to_mg(Context& ctx, int l, int nv, void* dst, const double* src, hipStream_t s) {
  Level& L = ctx.level(l);
  if (!ctx.ls) {
    MFMG_REQUIRE(&L == &ctx.levels.back(), MFMG_ERR_INVALID_ARG, "copy to the levels: finest level only");
    launch_cast(MFMG_F64, L.dtype, L.n_dofs * nv, src, dst, s);
    return;
  }
  MFMG_REQUIRE(&L != &ctx.active, MFMG_ERR_INVALID_ARG, "copy to the levels: not a multigrid level");
  launch_fill(0, dst, L.n_dofs * nv * static_cast<int64_t>(dtype_size(L.dtype)), s);
  launch_copy_map(MFMG_F64, L.dtype, L.n_copy, nv, L.cp_active.ptr, L.cp_level.ptr, src, dst, s);
}

void copy_from_mg(Context& ctx, int l, int nv, double* dst, const void* src, hipStream_t s) {
  Level& L = ctx.level(l);
  if (!ctx.ls) {
    MFMG_REQUIRE(&L == &ctx.levels.back(), MFMG_ERR_INVALID_ARG, "copy from the levels: finest level only");
    launch_cast(L.dtype, MFMG_F64, L.n_dofs * nv, src, dst, s);
    return;
  }
  MFMG_REQUIRE(&L != &ctx.active, MFMG_ERR_INVALID_ARG, "copy from the levels: not a multigrid level");
  launch_copy_map(L.dtype, MFMG_F64, L.n_copy, nv, L.cp_level.ptr, L.cp_active.ptr, src, dst, s);
}

void vcycle(Context& ctx, int nv, double* x, const double* b, hipStream_t s) {
  MFMG_REQUIRE(nv >= 1 && nv <= ctx.max_rhs, MFMG_ERR_INVALID_ARG, "n_vec exceeds max_rhs");
  if (ctx.ls) {  // Algorithm 1 over all levels, then the local-smoothing cycle
    const int nl = static_cast<int>(ctx.levels.size());
    for (int l = 0; l < nl; ++l) copy_to_mg(ctx, l, nv, ctx.levels[l].b.ptr, b, s);
    ls_vcycle_level(ctx, nl - 1, nv, s);
    for (int l = 0; l < nl; ++l) copy_from_mg(ctx, l, nv, x, ctx.levels[l].x.ptr, s);
    return;
  }
  Level& F = ctx.fine();
  const int64_t n = F.n_dofs * nv;
  launch_cast(MFMG_F64, F.dtype, n, b, F.b.ptr, s);  // copy_to_mg
  vcycle_level(ctx, static_cast<int>(ctx.levels.size()) - 1, nv, s);
  launch_cast(F.dtype, MFMG_F64, n, F.x.ptr, x, s);  // copy_from_mg
}

namespace {
// One V-cycle for the outer solver: eager, or replayed from a graph captured
// for this (x, b, n_vec) after a first eager run (which also initialises the
// launchers' one-time state outside the capture).
void solver_vcycle(Context& ctx, int nv, double* x, const double* b, hipStream_t s) {
  const NetState& N = ctx.net;
  if (!ctx.desc.graph_vcycle || N.mode != MFMG_COARSE_EXACT || N.rec_count < N.rec_capacity) {
    vcycle(ctx, nv, x, b, s);
    return;
  }
  GraphCache& G = ctx.graphs;
  for (const auto& e : G.entries)
    if (e.x == x && e.b == b && e.nv == nv) {
      MFMG_HIP(hipGraphLaunch(e.exec, s));
      return;
    }
  const GraphCache::Key key{x, b, nv};
  if (std::find(G.seen.begin(), G.seen.end(), key) == G.seen.end()) {
    G.seen.push_back(key);
    vcycle(ctx, nv, x, b, s);
    return;
  }
  if (!G.capture) MFMG_HIP(hipStreamCreateWithFlags(&G.capture, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  MFMG_HIP(hipStreamBeginCapture(G.capture, hipStreamCaptureModeThreadLocal));
  try {
    vcycle(ctx, nv, x, b, G.capture);
  } catch (...) {
    (void)hipStreamEndCapture(G.capture, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  MFMG_HIP(hipStreamEndCapture(G.capture, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  MFMG_HIP(err);
  G.entries.push_back({x, b, nv, exec});
  MFMG_HIP(hipGraphLaunch(exec, s));
}
}  // namespace

int pcg(Context& ctx, int nv, double* x, const double* b, double rtol, int max_it, bool flexible,
        mfmg_solve_stats* stats, hipStream_t s) {
  MFMG_REQUIRE(nv >= 1 && nv <= ctx.max_rhs, MFMG_ERR_INVALID_ARG, "n_vec exceeds max_rhs");
  Level& F = ctx.fine();
  const int64_t n = F.n_dofs;
  const int64_t nn = n * nv;
  double* sc = ctx.cg_scalar.ptr;  // [0..8) rz, [8..16) pq, [16..24) rr, [24..32) rz_new, [32..40) r.zold, [40..48) bb
  double* rz = sc;
  double* pq = sc + 8;
  double* rr = sc + 16;
  double* rzn = sc + 24;
  double* rzo = sc + 32;
  double* bb = sc + 40;
  hipEvent_t e0, e1;
  MFMG_HIP(hipEventCreate(&e0));
  MFMG_HIP(hipEventCreate(&e1));
  MFMG_HIP(hipEventRecord(e0, s));
  launch_fill(0, x, nn * 8, s);
  MFMG_HIP(hipMemcpyAsync(ctx.cg_r.ptr, b, nn * 8, hipMemcpyDeviceToDevice, s));
  launch_dot(n, nv, b, b, ctx.cg_partial.ptr, bb, s);
  std::vector<double> hb(nv), hr(nv);
  MFMG_HIP(hipMemcpyAsync(hb.data(), bb, nv * 8, hipMemcpyDeviceToHost, s));
  sync(s);
  for (int v = 0; v < nv; ++v) hb[v] = std::sqrt(hb[v]);
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->initial_residual = hb[0];
    stats->residual_history[0] = 1.0;
  }
  bool all_zero = true;
  for (int v = 0; v < nv; ++v) all_zero = all_zero && hb[v] == 0.0;
  int status = MFMG_ERR_NOT_CONVERGED;
  int it = 0;
  double worst = 0.0;
  if (all_zero) {
    status = MFMG_OK;
  } else {
    if (ctx.desc.fmg_start) {  // x0 from one full-multigrid pass, r0 = b - A x0
      fmg(ctx, nv, x, b, 1, s);
      launch_vmult(F.view, MFMG_F64, nv, ctx.cg_q.ptr, x, s);
      launch_residual_update(MFMG_F64, nn, b, ctx.cg_q.ptr, ctx.cg_r.ptr, s);
      launch_dot(n, nv, ctx.cg_r.ptr, ctx.cg_r.ptr, ctx.cg_partial.ptr, rr, s);
      MFMG_HIP(hipMemcpyAsync(hr.data(), rr, nv * 8, hipMemcpyDeviceToHost, s));
      sync(s);
      double w0 = 0.0;
      for (int v = 0; v < nv; ++v) w0 = std::max(w0, hb[v] > 0 ? std::sqrt(hr[v]) / hb[v] : 0.0);
      if (stats) stats->residual_history[0] = w0;
    }
    solver_vcycle(ctx, nv, ctx.cg_z.ptr, ctx.cg_r.ptr, s);
    MFMG_HIP(hipMemcpyAsync(ctx.cg_p.ptr, ctx.cg_z.ptr, nn * 8, hipMemcpyDeviceToDevice, s));
    launch_dot(n, nv, ctx.cg_r.ptr, ctx.cg_z.ptr, ctx.cg_partial.ptr, rz, s);
    for (it = 1; it <= max_it; ++it) {
      launch_vmult(F.view, MFMG_F64, nv, ctx.cg_q.ptr, ctx.cg_p.ptr, s);
      launch_dot(n, nv, ctx.cg_p.ptr, ctx.cg_q.ptr, ctx.cg_partial.ptr, pq, s);
      launch_cg_update_xr(n, nv, rz, pq, ctx.cg_p.ptr, ctx.cg_q.ptr, x, ctx.cg_r.ptr, s);
      launch_dot(n, nv, ctx.cg_r.ptr, ctx.cg_r.ptr, ctx.cg_partial.ptr, rr, s);
      std::vector<double> hpq(nv);
      MFMG_HIP(hipMemcpyAsync(hr.data(), rr, nv * 8, hipMemcpyDeviceToHost, s));
      MFMG_HIP(hipMemcpyAsync(hpq.data(), pq, nv * 8, hipMemcpyDeviceToHost, s));
      sync(s);
      worst = 0.0;
      bool breakdown = false;
      for (int v = 0; v < nv; ++v) {
        const double rel = hb[v] > 0 ? std::sqrt(hr[v]) / hb[v] : 0.0;
        worst = std::max(worst, rel);
        if (hb[v] > 0 && !(hpq[v] > 0.0) && rel > rtol) breakdown = true;
      }
      if (stats && it < 256) stats->residual_history[it] = worst;
      if (!std::isfinite(worst)) { status = MFMG_ERR_BREAKDOWN; break; }
      if (worst <= rtol) { status = MFMG_OK; break; }
      if (breakdown) { status = MFMG_ERR_BREAKDOWN; break; }
      if (flexible) std::swap(ctx.cg_z.ptr, ctx.cg_zold.ptr);
      solver_vcycle(ctx, nv, ctx.cg_z.ptr, ctx.cg_r.ptr, s);
      launch_dot(n, nv, ctx.cg_r.ptr, ctx.cg_z.ptr, ctx.cg_partial.ptr, rzn, s);
      if (flexible) launch_dot(n, nv, ctx.cg_r.ptr, ctx.cg_zold.ptr, ctx.cg_partial.ptr, rzo, s);
      launch_cg_update_p(n, nv, rzn, flexible ? rzo : nullptr, rz, ctx.cg_z.ptr, ctx.cg_p.ptr, s);
      MFMG_HIP(hipMemcpyAsync(rz, rzn, nv * 8, hipMemcpyDeviceToDevice, s));
    }
    if (it > max_it) it = max_it;
  }
  MFMG_HIP(hipEventRecord(e1, s));
  MFMG_HIP(hipEventSynchronize(e1));
  float ms = 0;
  MFMG_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (stats) {
    stats->iterations = it;
    stats->converged = status == MFMG_OK;
    stats->final_residual = worst;
    stats->time_ms = ms;
  }
  return status;
}

// The coefficient of every level from the finest level's cell values, on
// the device (the transfer of a cell field to the multigrid levels, Section
// 3.5): each coarser level's cells average the finer level's through the
// transfer's cell groups; then the cell masks, the diagonals and inverse
// diagonals, the Chebyshev intervals and the coarse direct solver follow the
// new operator, and captured V-cycles are dropped.
void set_coefficient(Context& ctx, const double* c_fine, hipStream_t s) {
  MFMG_REQUIRE(!ctx.ls, MFMG_ERR_UNSUPPORTED, "the coefficient update is built for global-coarsening levels");
  const int nl = static_cast<int>(ctx.levels.size());
  const Level& F = ctx.levels.back();
  {
    DeviceArray<int> flag(1);
    launch_fill(4, flag.ptr, 4, s);
    launch_coef_check(F.n_cells, c_fine, flag.ptr, s);
    int bad = 0;
    MFMG_HIP(hipMemcpyAsync(&bad, flag.ptr, 4, hipMemcpyDeviceToHost, s));
    sync(s);
    MFMG_REQUIRE(bad == 0, MFMG_ERR_INVALID_ARG, "the coefficient must lie in [1e-30, 1e30]");
  }
  std::vector<DeviceArray<double>> val(nl);
  const double* cur = c_fine;
  for (int l = nl - 1; l >= 0; --l) {
    Level& L = ctx.levels[l];
    if (l < nl - 1) {
      val[l].alloc(std::max<int64_t>(1, L.n_cells));
      launch_coef_restrict(ctx.levels[l + 1].tview, cur, val[l].ptr, s);
      cur = val[l].ptr;
    }
    launch_coef_apply(L.n_cells, cur, L.mask.ptr, L.meta.ptr, s);
    launch_diagonal(L.view, L.diag.ptr, s);
    launch_inverse_diag(MFMG_F64, L.n_dofs, L.diag.ptr, L.dinv.ptr, s);
    launch_inverse_diag(MFMG_F32, L.n_dofs, L.diag.ptr, L.dinv.ptr + L.n_dofs * 8, s);
  }
  sync(s);
  const mfmg_level_desc& desc = ctx.desc;
  const double range = desc.smoothing_range > 0 ? desc.smoothing_range : 20.0;
  const double safety = desc.eig_safety > 0 ? desc.eig_safety : 1.2;
  const int eig_it = desc.eig_iterations > 0 ? desc.eig_iterations : 15;
  for (int l = 1; l < nl; ++l) estimate_eigenvalues(ctx, ctx.levels[l], eig_it, safety, range, s);
  if (desc.dirichlet) {
    Level& L0 = ctx.levels[0];
    MFMG_HIP(hipMemcpyAsync(ctx.coarse_host.mask.data(), L0.mask.ptr, L0.n_cells * sizeof(uint32_t),
                            hipMemcpyDeviceToHost, s));
    sync(s);
    setup_coarse_solver(ctx);
  }
  ctx.graphs.clear();
  sync(s);
}

}  // namespace mfmg
