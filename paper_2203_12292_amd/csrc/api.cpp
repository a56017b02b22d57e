// extern "C" entry points (include/mfmg.h).
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "context.hpp"
#include "fe1d.hpp"
#include "net.hpp"

struct mfmg_ctx_s {
  mfmg::Context ctx;
};

// Work space of mfmg_vmult_noalloc: one file-scope device array per GPU the
// library runs on (it lives until the process ends).  Host code never passes
// the array's name to a kernel: it looks up the array's device address once
// per device and uses that.
#define MFMG_NOALLOC_SCRATCH_BYTES (64ll << 20)
static __device__ __align__(256) char scratch[MFMG_NOALLOC_SCRATCH_BYTES];

namespace {
thread_local std::string g_last_error;

// Device address of `scratch` on the current device, looked up on the first
// call on that device.
void* scratch_device_ptr() {
  static std::mutex mu;
  static std::vector<void*> ptrs;
  int dev = 0;
  MFMG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if (static_cast<int>(ptrs.size()) <= dev) ptrs.resize(dev + 1, nullptr);
  if (!ptrs[dev]) {
    void* p = nullptr;
    MFMG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    MFMG_REQUIRE(p != nullptr, MFMG_ERR_HIP, "no device address for the scratch array");
    ptrs[dev] = p;
  }
  return ptrs[dev];
}

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

template <typename F>
int guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const mfmg::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(MFMG_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(MFMG_ERR_INVALID_ARG, e.what());
  }
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

void check_dtype(int dt) {
  MFMG_REQUIRE(dt == MFMG_F64 || dt == MFMG_F32 || dt == MFMG_BF16, MFMG_ERR_UNSUPPORTED, "unknown dtype");
}

void check_ptr(const void* p, const char* name) {
  MFMG_REQUIRE(p != nullptr, MFMG_ERR_INVALID_ARG, std::string("null pointer: ") + name);
}

// a vector of n entries: NULL is accepted only when it is empty
void check_vec(const void* p, int64_t n, const char* name) {
  MFMG_REQUIRE(p != nullptr || n == 0, MFMG_ERR_INVALID_ARG, std::string("null pointer: ") + name);
}

void require_dirichlet(mfmg::Context& c) {
  MFMG_REQUIRE(c.desc.dirichlet != 0, MFMG_ERR_UNSUPPORTED,
               "the pure Neumann operator is singular: no coarse solve, V-cycle or solve");
}

void check_nv(mfmg::Context& c, int nv) {
  MFMG_REQUIRE(nv >= 1 && nv <= 8, MFMG_ERR_INVALID_ARG, "n_vec must be in [1, 8]");
  (void)c;
}
}  // namespace

extern "C" {

const char* mfmg_last_error(void) { return g_last_error.c_str(); }

int mfmg_setup_mesh(const mfmg_mesh_desc* desc, mfmg_mesh* out) {
  return guarded([&] {
    check_ptr(desc, "desc");
    check_ptr(out, "out");
    *out = nullptr;
    auto* m = new mfmg_mesh_s();
    try {
      m->gc.push_back(mfmg::build_octree(*desc));
      while (!m->gc.back().is_coarse_grid()) m->gc.push_back(m->gc.back().coarsened());
      std::reverse(m->gc.begin(), m->gc.end());  // index 0 = coarse grid
      int64_t nh = 0;
      for (const mfmg::Cell& c : m->gc.back().leaves()) nh += mfmg::leaf_has_hanging(m->gc.back(), c) ? 1 : 0;
      m->n_hanging_fine = nh;
    } catch (...) {
      delete m;
      throw;
    }
    *out = m;
    return MFMG_OK;
  });
}

int mfmg_mesh_info(mfmg_mesh mesh, int* n_meshes, int64_t* cells, int64_t* n_hanging_cells) {
  return guarded([&] {
    check_ptr(mesh, "mesh");
    if (n_meshes) *n_meshes = static_cast<int>(mesh->gc.size());
    if (cells)
      for (size_t i = 0; i < mesh->gc.size(); ++i) cells[i] = mesh->gc[i].n_leaves();
    if (n_hanging_cells) *n_hanging_cells = mesh->n_hanging_fine;
    return MFMG_OK;
  });
}

void mfmg_destroy_mesh(mfmg_mesh mesh) { delete mesh; }

int mfmg_host_level_matrix(mfmg_mesh mesh, int mesh_index, int degree, int dirichlet, int64_t* n_dofs,
                           int64_t* codes, double* dense) {
  return guarded([&] {
    check_ptr(mesh, "mesh");
    check_ptr(n_dofs, "n_dofs");
    MFMG_REQUIRE(mesh_index >= 0 && mesh_index < static_cast<int>(mesh->gc.size()), MFMG_ERR_INVALID_ARG,
                 "mesh index");
    mfmg::LevelDofs H = mfmg::build_level_dofs(mesh->gc[mesh_index], degree, dirichlet != 0, codes != nullptr);
    *n_dofs = H.n_dofs;
    if (codes) std::memcpy(codes, H.codes.data(), H.codes.size() * sizeof(int64_t));
    if (dense) {
      MFMG_REQUIRE(H.n_dofs <= 20000, MFMG_ERR_UNSUPPORTED, "dense matrix too large");
      std::vector<double> A = mfmg::assemble_dense(H, mfmg::Tables1D(degree));
      std::memcpy(dense, A.data(), A.size() * sizeof(double));
    }
    return MFMG_OK;
  });
}

int mfmg_host_ls_level(mfmg_mesh mesh, int level, int degree, int64_t* n_dofs, int64_t* n_copy, int64_t* codes,
                       uint8_t* edge, double* dense, int32_t* copy_level, int32_t* copy_active) {
  return guarded([&] {
    check_ptr(mesh, "mesh");
    check_ptr(n_dofs, "n_dofs");
    check_ptr(n_copy, "n_copy");
    const mfmg::Octree& tree = mesh->gc.back();
    MFMG_REQUIRE(level >= 0 && level <= tree.n_levels() && (level == 0 || !tree.refined[level - 1].empty()),
                 MFMG_ERR_INVALID_ARG, "refinement level without cells");
    mfmg::LevelDofs H = mfmg::build_level_dofs(tree, degree, true, codes != nullptr, level);
    mfmg::LevelDofs A = mfmg::build_level_dofs(tree, degree, true, false);
    std::vector<int32_t> cl, ca;
    mfmg::ls_copy_pairs(H, A, mfmg::EntityIndex(A), cl, ca);
    *n_dofs = H.n_dofs;
    *n_copy = static_cast<int64_t>(cl.size());
    if (codes) std::memcpy(codes, H.codes.data(), H.codes.size() * sizeof(int64_t));
    if (edge) std::memcpy(edge, H.dof_edge.data(), H.dof_edge.size());
    if (copy_level) std::memcpy(copy_level, cl.data(), cl.size() * sizeof(int32_t));
    if (copy_active) std::memcpy(copy_active, ca.data(), ca.size() * sizeof(int32_t));
    if (dense) {
      MFMG_REQUIRE(H.n_dofs <= 20000, MFMG_ERR_UNSUPPORTED, "dense matrix too large");
      std::vector<double> M = mfmg::assemble_dense(H, mfmg::Tables1D(degree));
      std::memcpy(dense, M.data(), M.size() * sizeof(double));
    }
    return MFMG_OK;
  });
}

int mfmg_setup_levels(mfmg_mesh mesh, const mfmg_level_desc* desc, void* stream, mfmg_ctx* out) {
  return guarded([&] {
    check_ptr(mesh, "mesh");
    check_ptr(desc, "desc");
    check_ptr(out, "out");
    *out = nullptr;
    auto* c = new mfmg_ctx_s();
    try {
      mfmg::setup_context(c->ctx, *mesh, *desc, as_stream(stream));
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
    return MFMG_OK;
  });
}

void mfmg_destroy_ctx(mfmg_ctx ctx) {
  if (ctx) {
    (void)hipDeviceSynchronize();
    delete ctx;
  }
}

int mfmg_n_levels(mfmg_ctx ctx, int* n_levels) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_ptr(n_levels, "n_levels");
    *n_levels = static_cast<int>(ctx->ctx.levels.size());
    return MFMG_OK;
  });
}

int mfmg_level_info(mfmg_ctx ctx, int level, int64_t* n_dofs, int64_t* n_cells, int* degree, int* dtype,
                    int64_t* n_hanging_cells) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    mfmg::Level& L = ctx->ctx.level(level);
    if (n_dofs) *n_dofs = L.n_dofs;
    if (n_cells) *n_cells = L.n_cells;
    if (degree) *degree = L.k;
    if (dtype) *dtype = L.dtype;
    if (n_hanging_cells) *n_hanging_cells = L.n_hanging;
    return MFMG_OK;
  });
}

int mfmg_level_dof_codes(mfmg_ctx ctx, int level, int64_t* codes) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_ptr(codes, "codes");
    mfmg::Level& L = ctx->ctx.level(level);
    mfmg::LevelDofs H =
        mfmg::build_level_dofs(ctx->ctx.meshes[L.mesh], L.k, ctx->ctx.desc.dirichlet != 0, true, L.only_level);
    MFMG_REQUIRE(H.n_dofs == L.n_dofs, MFMG_ERR_INVALID_ARG, "inconsistent level");
    std::memcpy(codes, H.codes.data(), H.codes.size() * sizeof(int64_t));
    return MFMG_OK;
  });
}

int mfmg_smoother_range(mfmg_ctx ctx, int level, double* lambda_min, double* lambda_max) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    mfmg::Level& L = ctx->ctx.level(level);
    if (lambda_min) *lambda_min = L.lmin;
    if (lambda_max) *lambda_max = L.lmax;
    return MFMG_OK;
  });
}

int mfmg_vmult(mfmg_ctx ctx, int level, int dtype, int n_vec, void* dst, const void* src, void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_dtype(dtype);
    check_nv(ctx->ctx, n_vec);
    mfmg::Level& L = ctx->ctx.level(level);
    MFMG_REQUIRE(n_vec <= ctx->ctx.max_rhs, MFMG_ERR_INVALID_ARG, "n_vec exceeds max_rhs");
    check_vec(dst, L.n_dofs, "dst");
    check_vec(src, L.n_dofs, "src");
    if (L.n_dofs == 0) return MFMG_OK;
    MFMG_REQUIRE(dst != src, MFMG_ERR_INVALID_ARG, "dst and src must not alias");
    if (dtype == MFMG_BF16) {
      mfmg::launch_vmult(L.view, dtype, n_vec, L.t.ptr, src, as_stream(stream));
      mfmg::launch_acc_to_storage(dtype, L.n_dofs * n_vec, L.t.ptr, dst, as_stream(stream));
    } else {
      mfmg::launch_vmult(L.view, dtype, n_vec, dst, src, as_stream(stream));
    }
    return MFMG_OK;
  });
}

int mfmg_vmult_noalloc(mfmg_ctx ctx, int level, int dtype, int n_vec, void* dst, const void* src, void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_dtype(dtype);
    check_nv(ctx->ctx, n_vec);
    mfmg::Level& L = ctx->ctx.level(level);
    check_vec(dst, L.n_dofs, "dst");
    check_vec(src, L.n_dofs, "src");
    if (L.n_dofs == 0) return MFMG_OK;
    MFMG_REQUIRE(dst != src, MFMG_ERR_INVALID_ARG, "dst and src must not alias");
    // scratch layout: the partial sums of the shared DoFs (arithmetic type),
    // then for bfloat16 the FP32 result before its rounding to the storage type
    const int64_t acc_bytes = dtype == MFMG_F64 ? 8 : 4;
    const int64_t part = (static_cast<int64_t>(L.sh_idx.n) * n_vec * acc_bytes + 255) / 256 * 256;
    const int64_t need = part + (dtype == MFMG_BF16 ? L.n_dofs * n_vec * 4 : 0);
    MFMG_REQUIRE(need <= MFMG_NOALLOC_SCRATCH_BYTES, MFMG_ERR_UNSUPPORTED,
                 "mfmg_vmult_noalloc: this level needs " + std::to_string(need) +
                     " bytes of work space, more than the " + std::to_string(MFMG_NOALLOC_SCRATCH_BYTES) +
                     " the library holds per GPU (use mfmg_vmult)");
    char* ws = static_cast<char*>(scratch_device_ptr());
    mfmg::CellView view = L.view;
    view.partial = ws;
    if (dtype == MFMG_BF16) {
      mfmg::launch_vmult(view, dtype, n_vec, ws + part, src, as_stream(stream));
      mfmg::launch_acc_to_storage(dtype, L.n_dofs * n_vec, ws + part, dst, as_stream(stream));
    } else {
      mfmg::launch_vmult(view, dtype, n_vec, dst, src, as_stream(stream));
    }
    return MFMG_OK;
  });
}

int mfmg_diagonal(mfmg_ctx ctx, int level, int dtype, void* diag, void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_dtype(dtype);
    mfmg::Level& L = ctx->ctx.level(level);
    check_vec(diag, L.n_dofs, "diag");
    if (L.n_dofs == 0) return MFMG_OK;
    if (dtype == MFMG_F64) {
      mfmg::launch_diagonal(L.view, static_cast<double*>(diag), as_stream(stream));
    } else {
      mfmg::launch_diagonal(L.view, reinterpret_cast<double*>(L.t.ptr), as_stream(stream));
      mfmg::launch_cast(MFMG_F64, dtype, L.n_dofs, L.t.ptr, diag, as_stream(stream));
    }
    return MFMG_OK;
  });
}

int mfmg_smooth(mfmg_ctx ctx, int level, int dtype, int n_vec, void* x, const void* b, int x_is_zero,
                const double* lambda, void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_dtype(dtype);
    mfmg::Level& L = ctx->ctx.level(level);
    MFMG_REQUIRE(n_vec >= 1 && n_vec <= ctx->ctx.max_rhs, MFMG_ERR_INVALID_ARG, "n_vec exceeds max_rhs");
    MFMG_REQUIRE(dtype == L.dtype, MFMG_ERR_INVALID_ARG, "dtype must equal the level's storage type");
    MFMG_REQUIRE(L.d.ptr != nullptr || L.n_dofs == 0, MFMG_ERR_UNSUPPORTED, "no smoother on the active mesh");
    check_vec(x, L.n_dofs, "x");
    check_vec(b, L.n_dofs, "b");
    double lmin = L.lmin, lmax = L.lmax;
    if (lambda) {
      lmin = lambda[0];
      lmax = lambda[1];
      MFMG_REQUIRE(lmax > lmin && lmin > 0, MFMG_ERR_INVALID_ARG, "need 0 < lambda_min < lambda_max");
    }
    if (L.n_dofs == 0) return MFMG_OK;
    mfmg::level_smooth(ctx->ctx, level, n_vec, x, b, x_is_zero != 0, lmin, lmax, as_stream(stream));
    return MFMG_OK;
  });
}

int mfmg_residual(mfmg_ctx ctx, int level, int dtype, int n_vec, void* r, const void* b, const void* x,
                  void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_dtype(dtype);
    mfmg::Level& L = ctx->ctx.level(level);
    MFMG_REQUIRE(n_vec >= 1 && n_vec <= ctx->ctx.max_rhs, MFMG_ERR_INVALID_ARG, "n_vec exceeds max_rhs");
    MFMG_REQUIRE(dtype == L.dtype, MFMG_ERR_INVALID_ARG, "dtype must equal the level's storage type");
    check_vec(r, L.n_dofs, "r");
    check_vec(b, L.n_dofs, "b");
    check_vec(x, L.n_dofs, "x");
    if (L.n_dofs == 0) return MFMG_OK;
    mfmg::level_residual(ctx->ctx, level, n_vec, r, b, x, as_stream(stream));
    return MFMG_OK;
  });
}

int mfmg_prolongate_add(mfmg_ctx ctx, int fine_level, int dtype, int n_vec, void* dst_fine, const void* src_coarse,
                        void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_dtype(dtype);
    check_nv(ctx->ctx, n_vec);
    MFMG_REQUIRE(fine_level >= 1, MFMG_ERR_INVALID_ARG, "fine level");
    const int64_t nf = ctx->ctx.level(fine_level).n_dofs, nc = ctx->ctx.level(fine_level - 1).n_dofs;
    check_vec(dst_fine, nf, "dst_fine");
    check_vec(src_coarse, nc, "src_coarse");
    if (nf == 0 || nc == 0) return MFMG_OK;
    mfmg::level_prolongate_add(ctx->ctx, fine_level, dtype, n_vec, dst_fine, src_coarse, as_stream(stream));
    return MFMG_OK;
  });
}

int mfmg_restrict_add(mfmg_ctx ctx, int fine_level, int dtype, int n_vec, void* dst_coarse, const void* src_fine,
                      void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_dtype(dtype);
    check_nv(ctx->ctx, n_vec);
    MFMG_REQUIRE(fine_level >= 1, MFMG_ERR_INVALID_ARG, "fine level");
    const int64_t nf = ctx->ctx.level(fine_level).n_dofs, nc = ctx->ctx.level(fine_level - 1).n_dofs;
    check_vec(src_fine, nf, "src_fine");
    check_vec(dst_coarse, nc, "dst_coarse");
    if (nf == 0 || nc == 0) return MFMG_OK;
    mfmg::level_restrict_add(ctx->ctx, fine_level, dtype, n_vec, dst_coarse, src_fine, as_stream(stream));
    return MFMG_OK;
  });
}

int mfmg_coarse_solve(mfmg_ctx ctx, int dtype, int n_vec, void* x, const void* b, void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_dtype(dtype);
    check_nv(ctx->ctx, n_vec);
    require_dirichlet(ctx->ctx);
    check_vec(x, ctx->ctx.n0, "x");
    check_vec(b, ctx->ctx.n0, "b");
    if (ctx->ctx.n0 == 0) return MFMG_OK;
    mfmg::coarse_solve(ctx->ctx, dtype, n_vec, x, b, as_stream(stream));
    return MFMG_OK;
  });
}

int mfmg_vcycle(mfmg_ctx ctx, int n_vec, void* x_f64, const void* b_f64, void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    require_dirichlet(ctx->ctx);
    check_vec(x_f64, ctx->ctx.fine().n_dofs, "x");
    check_vec(b_f64, ctx->ctx.fine().n_dofs, "b");
    if (ctx->ctx.fine().n_dofs == 0) return MFMG_OK;
    mfmg::vcycle(ctx->ctx, n_vec, static_cast<double*>(x_f64), static_cast<const double*>(b_f64),
                 as_stream(stream));
    return MFMG_OK;
  });
}

int mfmg_fmg(mfmg_ctx ctx, int n_vec, void* x_f64, const void* b_f64, int cycles, void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    require_dirichlet(ctx->ctx);
    check_vec(x_f64, ctx->ctx.fine().n_dofs, "x");
    check_vec(b_f64, ctx->ctx.fine().n_dofs, "b");
    if (ctx->ctx.fine().n_dofs == 0) return MFMG_OK;
    mfmg::fmg(ctx->ctx, n_vec, static_cast<double*>(x_f64), static_cast<const double*>(b_f64), cycles,
              as_stream(stream));
    return MFMG_OK;
  });
}

int mfmg_copy_to_mg(mfmg_ctx ctx, int level, int n_vec, void* dst, const void* src_f64, void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    MFMG_REQUIRE(n_vec >= 1 && n_vec <= ctx->ctx.max_rhs, MFMG_ERR_INVALID_ARG, "n_vec exceeds max_rhs");
    mfmg::Level& L = ctx->ctx.level(level);
    check_vec(dst, L.n_dofs, "dst");
    check_vec(src_f64, ctx->ctx.fine().n_dofs, "src");
    if (L.n_dofs == 0) return MFMG_OK;
    mfmg::copy_to_mg(ctx->ctx, level, n_vec, dst, static_cast<const double*>(src_f64), as_stream(stream));
    return MFMG_OK;
  });
}

int mfmg_copy_from_mg(mfmg_ctx ctx, int level, int n_vec, void* dst_f64, const void* src, void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    MFMG_REQUIRE(n_vec >= 1 && n_vec <= ctx->ctx.max_rhs, MFMG_ERR_INVALID_ARG, "n_vec exceeds max_rhs");
    mfmg::Level& L = ctx->ctx.level(level);
    check_vec(src, L.n_dofs, "src");
    check_vec(dst_f64, ctx->ctx.fine().n_dofs, "dst");
    if (L.n_dofs == 0) return MFMG_OK;
    mfmg::copy_from_mg(ctx->ctx, level, n_vec, static_cast<double*>(dst_f64), src, as_stream(stream));
    return MFMG_OK;
  });
}

int mfmg_level_edge(mfmg_ctx ctx, int level, int64_t* n_edge, uint8_t* flags) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    mfmg::Level& L = ctx->ctx.level(level);
    if (n_edge) *n_edge = L.n_edge;
    if (flags) {
      if (L.host_edge.empty()) std::memset(flags, 0, static_cast<size_t>(L.n_dofs));
      else std::memcpy(flags, L.host_edge.data(), L.host_edge.size());
    }
    return MFMG_OK;
  });
}

int mfmg_solve(mfmg_ctx ctx, int n_vec, void* x_f64, const void* b_f64, double rtol, int max_it, int flexible,
               mfmg_solve_stats* stats, void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    require_dirichlet(ctx->ctx);
    check_vec(x_f64, ctx->ctx.fine().n_dofs, "x");
    check_vec(b_f64, ctx->ctx.fine().n_dofs, "b");
    MFMG_REQUIRE(rtol > 0 && max_it >= 0, MFMG_ERR_INVALID_ARG, "rtol must be > 0, max_it >= 0");
    if (ctx->ctx.fine().n_dofs == 0) {
      if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->converged = 1;
      }
      return static_cast<int>(MFMG_OK);
    }
    int st = mfmg::pcg(ctx->ctx, n_vec, static_cast<double*>(x_f64), static_cast<const double*>(b_f64), rtol,
                       max_it, flexible != 0, stats, as_stream(stream));
    if (st == MFMG_ERR_NOT_CONVERGED) g_last_error = "PCG did not converge within max_it";
    if (st == MFMG_ERR_BREAKDOWN) g_last_error = "PCG breakdown (p^T A p <= 0 or non-finite residual)";
    return st;
  });
}

int mfmg_rhs(mfmg_ctx ctx, int level, int kind, const double* params, int n_terms, int n_vec, void* b_f64,
             void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_ptr(params, "params");
    check_nv(ctx->ctx, n_vec);
    MFMG_REQUIRE(kind == MFMG_RHS_CONST || kind == MFMG_RHS_GAUSS || kind == MFMG_RHS_SINE, MFMG_ERR_INVALID_ARG,
                 "rhs kind");
    MFMG_REQUIRE(kind != MFMG_RHS_GAUSS || n_terms >= 1, MFMG_ERR_INVALID_ARG, "n_terms");
    mfmg::Level& L = ctx->ctx.level(level);
    check_vec(b_f64, L.n_dofs, "b");
    if (L.n_dofs == 0) return MFMG_OK;
    const size_t np = kind == MFMG_RHS_CONST ? 1 : kind == MFMG_RHS_SINE ? 2 : static_cast<size_t>(n_terms) * 5 * n_vec;
    mfmg::DeviceArray<double>& dp = ctx->ctx.rhs_params;
    MFMG_HIP(hipStreamSynchronize(as_stream(stream)));  // a previous load may still read dp
    if (dp.n < np) dp.alloc(np);
    MFMG_HIP(hipMemcpyAsync(dp.ptr, params, np * sizeof(double), hipMemcpyHostToDevice, as_stream(stream)));
    mfmg::launch_rhs(L.view, kind, dp.ptr, kind == MFMG_RHS_GAUSS ? n_terms : 0, n_vec,
                     static_cast<double*>(b_f64), as_stream(stream));
    MFMG_HIP(hipStreamSynchronize(as_stream(stream)));
    return MFMG_OK;
  });
}

int mfmg_distribute(mfmg_ctx ctx, int level, const void* x_f64, void* out_f64, void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_ptr(out_f64, "out");
    mfmg::Level& L = ctx->ctx.level(level);
    check_vec(x_f64, L.n_dofs, "x");
    mfmg::launch_distribute(L.view, static_cast<const double*>(x_f64), static_cast<double*>(out_f64),
                            as_stream(stream));
    return MFMG_OK;
  });
}

int mfmg_level_cells(mfmg_ctx ctx, int level, int32_t* levels, int32_t* ijk) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    mfmg::Level& L = ctx->ctx.level(level);
    if (levels) std::memcpy(levels, L.host_levels.data(), L.host_levels.size() * sizeof(int32_t));
    if (ijk) std::memcpy(ijk, L.host_ijk.data(), L.host_ijk.size() * sizeof(int32_t));
    return MFMG_OK;
  });
}

static void require_net(mfmg::Context& c) {
  MFMG_REQUIRE(c.net.n_params > 0, MFMG_ERR_UNSUPPORTED,
               "learned coarse correction needs a coarse level without hanging nodes, <= 2048 DoFs and "
               "degree <= 2");
}

int mfmg_net_n_params(mfmg_ctx ctx, int* n) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_ptr(n, "n");
    require_net(ctx->ctx);
    *n = ctx->ctx.net.n_params;
    return MFMG_OK;
  });
}

int mfmg_net_record(mfmg_ctx ctx, int capacity) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    require_net(ctx->ctx);
    MFMG_REQUIRE(capacity >= 0, MFMG_ERR_INVALID_ARG, "capacity must be >= 0");
    mfmg::NetState& N = ctx->ctx.net;
    MFMG_HIP(hipDeviceSynchronize());
    N.rec_capacity = capacity;
    N.rec_count = 0;
    if (capacity == 0) N.record.release();
    else N.record.alloc(static_cast<size_t>(capacity) * N.n0);
    return MFMG_OK;
  });
}

int mfmg_net_n_recorded(mfmg_ctx ctx, int* n) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_ptr(n, "n");
    *n = ctx->ctx.net.rec_count;
    return MFMG_OK;
  });
}

int mfmg_net_set_params(mfmg_ctx ctx, const float* theta, int n) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_ptr(theta, "theta");
    require_net(ctx->ctx);
    MFMG_REQUIRE(n == ctx->ctx.net.n_params, MFMG_ERR_INVALID_ARG, "parameter count");
    MFMG_HIP(hipMemcpy(ctx->ctx.net.params.ptr, theta, n * sizeof(float), hipMemcpyHostToDevice));
    return MFMG_OK;
  });
}

int mfmg_net_get_params(mfmg_ctx ctx, float* theta, int n) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_ptr(theta, "theta");
    require_net(ctx->ctx);
    MFMG_REQUIRE(n == ctx->ctx.net.n_params, MFMG_ERR_INVALID_ARG, "parameter count");
    MFMG_HIP(hipMemcpy(theta, ctx->ctx.net.params.ptr, n * sizeof(float), hipMemcpyDeviceToHost));
    return MFMG_OK;
  });
}

int mfmg_net_loss_grad(mfmg_ctx ctx, int n_rows, const float* X, const float* T, float* grad, float* loss) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_ptr(X, "X");
    check_ptr(T, "T");
    check_ptr(grad, "grad");
    require_net(ctx->ctx);
    MFMG_REQUIRE(n_rows > 0, MFMG_ERR_INVALID_ARG, "n_rows must be > 0");
    float l = mfmg::net_loss_grad(ctx->ctx, n_rows, X, T, grad, ctx->ctx.stream);
    if (loss) *loss = l;
    return MFMG_OK;
  });
}

int mfmg_net_train(mfmg_ctx ctx, const mfmg_net_train_desc* desc, float* history) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_ptr(desc, "desc");
    require_net(ctx->ctx);
    MFMG_REQUIRE(desc->epochs >= 1 && desc->batch_rows >= 0, MFMG_ERR_INVALID_ARG, "epochs/batch_rows");
    mfmg::net_train(ctx->ctx, *desc, history, ctx->ctx.stream);
    MFMG_HIP(hipStreamSynchronize(ctx->ctx.stream));
    return MFMG_OK;
  });
}

int mfmg_set_coefficient(mfmg_ctx ctx, const void* c_f64, void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_vec(c_f64, ctx->ctx.levels.empty() ? 0 : ctx->ctx.levels.back().n_cells, "c");
    mfmg::set_coefficient(ctx->ctx, static_cast<const double*>(c_f64), as_stream(stream));
    return MFMG_OK;
  });
}

int mfmg_net_infer(mfmg_ctx ctx, int dtype, void* y, const void* b, void* stream) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    check_dtype(dtype);
    require_net(ctx->ctx);
    check_vec(y, ctx->ctx.n0, "y");
    check_vec(b, ctx->ctx.n0, "b");
    MFMG_REQUIRE(y != b, MFMG_ERR_INVALID_ARG, "y and b must not alias");
    mfmg::net_predict(ctx->ctx, dtype, y, b, as_stream(stream));
    return MFMG_OK;
  });
}

int mfmg_net_mode(mfmg_ctx ctx, int mode, double tau) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    MFMG_REQUIRE(mode == MFMG_COARSE_EXACT || mode == MFMG_COARSE_LEARNED || mode == MFMG_COARSE_ZERO,
                 MFMG_ERR_INVALID_ARG, "coarse mode");
    if (mode != MFMG_COARSE_EXACT) require_net(ctx->ctx);
    MFMG_REQUIRE(tau >= 0, MFMG_ERR_INVALID_ARG, "tau must be >= 0");
    ctx->ctx.net.mode = mode;
    ctx->ctx.net.tau = tau;
    return MFMG_OK;
  });
}

int mfmg_net_counts(mfmg_ctx ctx, int* accepted, int* rejected, double* mean_rel_residual) {
  return guarded([&] {
    check_ptr(ctx, "ctx");
    require_net(ctx->ctx);
    int c[2] = {0, 0};
    MFMG_HIP(hipDeviceSynchronize());
    MFMG_HIP(hipMemcpy(c, ctx->ctx.net.counters.ptr, 8, hipMemcpyDeviceToHost));
    double rs = 0.0;
    MFMG_HIP(hipMemcpy(&rs, ctx->ctx.net.relsum.ptr, 8, hipMemcpyDeviceToHost));
    MFMG_HIP(hipMemset(ctx->ctx.net.counters.ptr, 0, 8));
    MFMG_HIP(hipMemset(ctx->ctx.net.relsum.ptr, 0, 8));
    if (accepted) *accepted = c[0];
    if (rejected) *rejected = c[1];
    if (mean_rel_residual) *mean_rel_residual = (c[0] + c[1]) > 0 ? rs / (c[0] + c[1]) : 0.0;
    return MFMG_OK;
  });
}

}  // extern "C"
