// Device kernels of the matrix-free multigrid hot path (CDNA4 / gfx950).
//
// Cell operator (Eq. impl:mf): v = sum_e G_e^T C_e^T S_e^T Q_e S_e C_e G_e x.
// Every cell is an axis-aligned cube of side h, so the quadrature-point
// operation Q_e reduces to the scalar h * w_q and the cell matrix has the
// tensor form h (K (x) M (x) M + M (x) K (x) M + M (x) M (x) K) with the 1D
// mass M and stiffness K integrated exactly by the (k+1)-point Gauss rule.
// The kernel applies it as seven 1D sweeps: M_x/K_x, then M_y/K_y, then
// M_z/K_z (fewer contractions than interpolating to quadrature points and
// back, same result up to rounding).
//
// Thread layout: n^2 threads per cell (n = k+1), each owning one line of n
// nodes; a block holds CPB cells.  A phase works on lines along one axis in
// registers; LDS re-distributes the cell's n^3 values between phases.
// Hanging-node constraints (Section 3.2, the in-place interpolation variant)
// are 1D interpolations along the lines of the hanging faces/edges, applied
// in the phase whose lines run along that axis: gather + z, y, x before the
// operator, transposed z, x, y after it, then the scatter.
#include "common.hpp"
#include "fe1d.hpp"
#include "geometry.hpp"
#include "kernels.hpp"
#include "slots.hpp"

namespace mfmg {

// ---------------------------------------------------------------------------
// tables passed by value as kernel arguments (scalar-loaded)
template <typename T, int N>
struct OpTab {
  T M[N * N];
  T K[N * N];
  T H[2][N * N];
};

// A symmetric, centrosymmetric n x n matrix (the 1D mass and stiffness
// matrices on Gauss-Lobatto nodes) in even-odd form: with h = n/2,
// e_j = x_j + x_{n-1-j}, o_j = x_j - x_{n-1-j} (j < h),
//   y_i       = sum_j E_ij e_j + c_i x_h + sum_j O_ij o_j      (i < h)
//   y_{n-1-i} = sum_j E_ij e_j + c_i x_h - sum_j O_ij o_j
//   y_h       = sum_j c_j e_j + d x_h                          (n odd)
// where E = (A_ij + A_i,n-1-j)/2 and O = (A_ij - A_i,n-1-j)/2 are symmetric
// (upper triangles stored), c_i = A_ih, d = A_hh.
template <typename T, int N>
struct SymMat {
  static constexpr int H = N / 2;
  static constexpr int NE = H * (H + 1) / 2;
  T e[NE > 0 ? NE : 1];
  T o[NE > 0 ? NE : 1];
  T c[H > 0 ? H : 1];
  T d;
};

__host__ __device__ constexpr int sym_idx(int i, int j, int h) {
  return i <= j ? i * h - i * (i - 1) / 2 + (j - i) : j * h - j * (j - 1) / 2 + (i - j);
}

// Operator tables: mass and stiffness in even-odd form (kernel arguments,
// scalar registers) and the hanging-node interpolation (copied to LDS).
template <typename T, int N>
struct OpTab2 {
  SymMat<T, N> M, K;
  T Hg[2 * N * N];  // [s][i][j] = l_j((s + xi_i)/2)
};

template <typename T, int NF, int NC>
struct TrTab {
  T P[NF * NC];     // 1D prolongation, row-major NF x NC
  T H[2][NC * NC];  // hanging interpolation of the coarse cell
};

template <int N>
struct Gauss1D {
  double x[N];      // Gauss points on [0, 1]
  double w[N];      // weights
  double S[N * N];  // S[q*N + i] = l_i(x_q)
};

inline const Tables1D& tables(int k) {
  static Tables1D t[7] = {Tables1D(1), Tables1D(1), Tables1D(2), Tables1D(3),
                          Tables1D(4), Tables1D(5), Tables1D(6)};
  return t[k];
}

template <int N>
Gauss1D<N> make_gauss() {
  const Tables1D& t = tables(N - 1);
  Gauss1D<N> g;
  for (int i = 0; i < N; ++i) {
    g.x[i] = t.qp[i];
    g.w[i] = t.qw[i];
  }
  for (int i = 0; i < N * N; ++i) g.S[i] = t.S[i];
  return g;
}

template <typename T, int N>
OpTab<T, N> make_optab() {
  const Tables1D& t = tables(N - 1);
  OpTab<T, N> o;
  for (int i = 0; i < N * N; ++i) {
    o.M[i] = static_cast<T>(t.M[i]);
    o.K[i] = static_cast<T>(t.K[i]);
    o.H[0][i] = static_cast<T>(t.H[0][i]);
    o.H[1][i] = static_cast<T>(t.H[1][i]);
  }
  return o;
}

template <typename T, int N>
SymMat<T, N> make_sym(const std::vector<double>& A) {
  SymMat<T, N> m{};
  constexpr int H = N / 2;
  for (int i = 0; i < H; ++i)
    for (int j = i; j < H; ++j) {
      m.e[sym_idx(i, j, H)] = static_cast<T>(0.5 * (A[i * N + j] + A[i * N + (N - 1 - j)]));
      m.o[sym_idx(i, j, H)] = static_cast<T>(0.5 * (A[i * N + j] - A[i * N + (N - 1 - j)]));
    }
  if (N % 2) {
    for (int i = 0; i < H; ++i) m.c[i] = static_cast<T>(A[i * N + H]);
    m.d = static_cast<T>(A[H * N + H]);
  }
  return m;
}

template <typename T, int N>
OpTab2<T, N> make_optab2() {
  const Tables1D& t = tables(N - 1);
  OpTab2<T, N> o;
  o.M = make_sym<T, N>(t.M);
  o.K = make_sym<T, N>(t.K);
  for (int i = 0; i < N * N; ++i) {
    o.Hg[i] = static_cast<T>(t.H[0][i]);
    o.Hg[N * N + i] = static_cast<T>(t.H[1][i]);
  }
  return o;
}

// The hanging interpolation matrices of both halves in constant memory, for
// wavefronts holding one cell: read with uniform addresses, they become
// scalar loads and scalar operands.  Filled once per device before the first
// operator launch that uses them.
template <typename T, int N>
struct HgTable {
  T v[2 * N * N];
};
template <typename T, int N>
__constant__ HgTable<T, N> kHgTab;

template <typename T, int N>
void ensure_hg_table() {
  static bool done[64] = {};
  int dev = 0;
  MFMG_HIP(hipGetDevice(&dev));
  MFMG_REQUIRE(dev >= 0 && dev < 64, MFMG_ERR_UNSUPPORTED, "device index");
  if (done[dev]) return;
  const OpTab2<T, N> o = make_optab2<T, N>();
  MFMG_HIP(hipMemcpyToSymbol(HIP_SYMBOL((kHgTab<T, N>)), o.Hg, sizeof(o.Hg)));
  done[dev] = true;
}

// y = A x for a SymMat A (even-odd evaluation)
template <int N, typename T>
__device__ __forceinline__ void sym_mv(const SymMat<T, N>& A, const T (&x)[N], T (&y)[N]) {
  constexpr int H = N / 2;
  T e[H > 0 ? H : 1], o[H > 0 ? H : 1];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    e[j] = x[j] + x[N - 1 - j];
    o[j] = x[j] - x[N - 1 - j];
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    T se = A.e[sym_idx(i, 0, H)] * e[0];
    T so = A.o[sym_idx(i, 0, H)] * o[0];
#pragma unroll
    for (int j = 1; j < H; ++j) {
      se += A.e[sym_idx(i, j, H)] * e[j];
      so += A.o[sym_idx(i, j, H)] * o[j];
    }
    if constexpr (N % 2 == 1) se += A.c[i] * x[H];
    y[i] = se + so;
    y[N - 1 - i] = se - so;
  }
  if constexpr (N % 2 == 1) {
    T m = A.d * x[H];
#pragma unroll
    for (int j = 0; j < H; ++j) m += A.c[j] * e[j];
    y[H] = m;
  }
}

// In-place hanging interpolation of a line from the LDS table Hg (both
// halves, [s][i][j]): u <- H_s u (H_s^T u if TRANS).
template <int N, typename T, bool TRANS>
__device__ __forceinline__ void interp_lds(const T* __restrict__ Hg, int s, T (&u)[N]) {
  const T* Hs = Hg + s * N * N;
  T out[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < N; ++j) acc += Hs[TRANS ? j * N + i : i * N + j] * u[j];
    out[i] = acc;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] = out[i];
}

// The same from the constant-memory table when s is the same on every lane
// of the wavefront (one cell per wavefront): the branch is uniform and the
// table entries are scalar operands, no LDS reads.
template <int N, typename T, bool TRANS, int S>
__device__ __forceinline__ void interp_const(T (&u)[N]) {
  // an opaque copy of the table address keeps the loads here, next to their
  // use (hoisted out of the cell loop, 2 x N^2 values would not fit the
  // scalar registers)
  using CT = const __attribute__((address_space(4))) T;
  CT* tbl = reinterpret_cast<CT*>(reinterpret_cast<uintptr_t>(kHgTab<T, N>.v)) + S * N * N;
  asm volatile("" : "+s"(tbl));
  T out[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < N; ++j) acc += tbl[TRANS ? j * N + i : i * N + j] * u[j];
    out[i] = acc;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] = out[i];
}

// u <- H_s u (H_s^T u if TRANS) for the hanging lines of a cell, from the
// constant-memory table.  UNI: s is wavefront-uniform, a uniform branch picks
// the half.  Otherwise s differs between the cells of a wavefront: the halves
// are mirror images, H_1 = J H_0 J with J the reversal of the node order (the
// nodes are symmetric about the midpoint and l_j(1 - t) = l_{n-1-j}(t)), so
// each lane reverses its line where s = 1, applies H_0 (scalar operands) and
// reverses back: 2n selects instead of n^2 LDS reads of the table.
template <int N, typename T, bool TRANS, bool UNI>
__device__ __forceinline__ void hang_interp(const T* __restrict__ Hg, int s, T (&u)[N]) {
  (void)Hg;
  if constexpr (UNI) {
    if (s) interp_const<N, T, TRANS, 1>(u);
    else interp_const<N, T, TRANS, 0>(u);
  } else {
    T w[N];
#pragma unroll
    for (int j = 0; j < N; ++j) w[j] = s ? u[N - 1 - j] : u[j];
    interp_const<N, T, TRANS, 0>(w);
#pragma unroll
    for (int i = 0; i < N; ++i) u[i] = s ? w[N - 1 - i] : w[i];
  }
}

// ---------------------------------------------------------------------------
// small dense 1D contractions on register arrays
template <int N, typename T>
__device__ __forceinline__ void mv(const T* __restrict__ A, const T (&x)[N], T (&y)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = A[i * N] * x[0];
#pragma unroll
    for (int j = 1; j < N; ++j) s += A[i * N + j] * x[j];
    y[i] = s;
  }
}

// y = A x + B z (A, B symmetric use)
template <int N, typename T>
__device__ __forceinline__ void mv2(const T* __restrict__ A, const T (&x)[N], const T* __restrict__ B,
                                    const T (&z)[N], T (&y)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = A[i * N] * x[0];
#pragma unroll
    for (int j = 1; j < N; ++j) s += A[i * N + j] * x[j];
#pragma unroll
    for (int j = 0; j < N; ++j) s += B[i * N + j] * z[j];
    y[i] = s;
  }
}

// in-place hanging interpolation u <- H_s u (transpose: u <- H_s^T u)
template <int N, typename T, bool TRANS>
__device__ __forceinline__ void interp(const T (&H)[2][N * N], int s, T (&u)[N]) {
  T out[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int idx = TRANS ? j * N + i : i * N + j;
      const T h = s ? H[1][idx] : H[0][idx];
      acc += h * u[j];
    }
    out[i] = acc;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] = out[i];
}

template <typename T> __device__ __forceinline__ void atomic_add(T* p, T v) { unsafeAtomicAdd(p, v); }

// bfloat16 add through a compare-and-swap on the enclosing 32-bit word
// (used only on the small levels stored in bfloat16)
__device__ __forceinline__ void atomic_add_bf16(bf16* p, float v) {
  uintptr_t addr = reinterpret_cast<uintptr_t>(p);
  unsigned int* word = reinterpret_cast<unsigned int*>(addr & ~uintptr_t(3));
  const unsigned int shift = (addr & 2) ? 16u : 0u;
  unsigned int old = *word, assumed;
  do {
    assumed = old;
    bf16 cur;
    cur.bits = static_cast<uint16_t>((assumed >> shift) & 0xffffu);
    bf16 nv = float_to_bf16(bf16_to_float(cur) + v);
    unsigned int repl = (assumed & ~(0xffffu << shift)) | (static_cast<unsigned int>(nv.bits) << shift);
    old = atomicCAS(word, assumed, repl);
  } while (old != assumed);
}

// dst += v for a storage-typed vector entry; `exclusive` entries have no
// concurrent writer and use a plain read-modify-write.
template <typename S, typename T>
__device__ __forceinline__ void add_to(S* p, T v, bool exclusive) {
  if (exclusive) {
    *p = store_as<S>(load_as<T>(*p) + v);
  } else {
    if constexpr (sizeof(S) == 2) atomic_add_bf16(reinterpret_cast<bf16*>(p), static_cast<float>(v));
    else atomic_add(p, static_cast<S>(v));
  }
}

// scatter-add of the line of nodes (a, 0..k, c) (along y); cell interiors are
// owned by the cell (plain store), shared entities use atomics.
// `plain`: no other cell writes the same entities concurrently (deterministic
// mode, colour by colour), a plain read-modify-write.
template <typename T>
__device__ __forceinline__ void scatter_add(T* p, T v, bool plain) {
  if (plain) *p += v;
  else atomic_add(p, v);
}

template <int K, typename T>
__device__ __forceinline__ void scatter_yline(const int32_t* __restrict__ ent, int64_t nc, int64_t cell,
                                              int a, int c, const T (&w)[K + 1], T* __restrict__ dst, int nv,
                                              int v, bool plain = false) {
  const int s0 = node_slot(a, 0, c, K), s1 = node_slot(a, K, c, K);
  const int o0 = node_offset(a, 0, c, K);
  const int32_t e0 = ent[s0 * nc + cell], e1 = ent[s1 * nc + cell];
  if (e0 >= 0) scatter_add(&dst[static_cast<int64_t>(e0 + o0) * nv + v], w[0], plain);
  if (e1 >= 0) scatter_add(&dst[static_cast<int64_t>(e1 + o0) * nv + v], w[K], plain);
  if constexpr (K > 1) {
    const int sm = node_slot(a, 1, c, K);
    const int om = node_offset(a, 1, c, K);
    const int st = K > 2 ? node_offset(a, 2, c, K) - om : 0;
    const int32_t em = ent[sm * nc + cell];
    if (em >= 0) {
      if (sm == 26) {
#pragma unroll
        for (int b = 1; b < K; ++b) dst[static_cast<int64_t>(em + om + (b - 1) * st) * nv + v] = w[b];
      } else {
#pragma unroll
        for (int b = 1; b < K; ++b)
          scatter_add(&dst[static_cast<int64_t>(em + om + (b - 1) * st) * nv + v], w[b], plain);
      }
    }
  }
}

// Barrier of the cell pipeline.  All lanes of a cell belong to one
// wavefront and LDS operations of a wavefront execute in order, so a compiler
// code-motion barrier with wavefront-scope fences is enough.
struct WaveSync {
  __device__ __forceinline__ void operator()() const {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
};

// The cell pipeline C^T S^T Q S C on the block's LDS.  Input: this thread's
// z-line (x = ta, y = tb) of gathered slot values.  Output: this thread's
// y-line (x = ta, z = tb) of the result, before the scatter.  Must be called
// by all threads of the block (contains barriers).
template <int K, typename T, typename Sync>
__device__ __forceinline__ void cell_pipeline(T* __restrict__ B0, T* __restrict__ B1, bool active, uint32_t m,
                                              int block_hang, T h, const OpTab<T, K + 1>& tab, int ta, int tb,
                                              T (&u)[K + 1]) {
  const Sync sync{};
  constexpr int N = K + 1, N2 = N * N;
  const bool hang = mask_hanging(m);
  // phase 1: z-lines (x = ta, y = tb): hanging z-interpolation, store
  if (active) {
    if (hang && hanging_line(m, 2, ta, tb, K)) interp<N, T, false>(tab.H, mask_sub(m, 2), u);
#pragma unroll
    for (int c = 0; c < N; ++c) B0[c * N2 + tb * N + ta] = u[c];
  }
  sync();
  // phase 2: y-lines (x = ta, z = tb): hanging y-interpolation
  if (block_hang) {
    if (active && hang && hanging_line(m, 1, ta, tb, K)) {
#pragma unroll
      for (int r = 0; r < N; ++r) u[r] = B0[tb * N2 + r * N + ta];
      interp<N, T, false>(tab.H, mask_sub(m, 1), u);
#pragma unroll
      for (int r = 0; r < N; ++r) B0[tb * N2 + r * N + ta] = u[r];
    }
    sync();
  }
  // phase 3: x-lines (y = ta, z = tb): hanging x-interpolation, M_x, K_x
  T a[N], b[N];
  if (active) {
#pragma unroll
    for (int r = 0; r < N; ++r) u[r] = B0[tb * N2 + ta * N + r];
    if (hang && hanging_line(m, 0, ta, tb, K)) interp<N, T, false>(tab.H, mask_sub(m, 0), u);
    mv<N>(tab.M, u, a);
    mv<N>(tab.K, u, b);
#pragma unroll
    for (int r = 0; r < N; ++r) {
      B0[tb * N2 + ta * N + r] = a[r];
      B1[tb * N2 + ta * N + r] = b[r];
    }
  }
  sync();
  // phase 4: y-lines (x = ta, z = tb): M_y a ; K_y a + M_y b
  if (active) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      a[r] = B0[tb * N2 + r * N + ta];
      b[r] = B1[tb * N2 + r * N + ta];
    }
    T c1[N], f[N];
    mv<N>(tab.M, a, c1);
    mv2<N>(tab.K, a, tab.M, b, f);
#pragma unroll
    for (int r = 0; r < N; ++r) {
      B0[tb * N2 + r * N + ta] = c1[r];
      B1[tb * N2 + r * N + ta] = f[r];
    }
  }
  sync();
  // phase 5: z-lines (x = ta, y = tb): h (K_z c + M_z f), transposed z-interpolation
  if (active) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      a[r] = B0[r * N2 + tb * N + ta];
      b[r] = B1[r * N2 + tb * N + ta];
    }
    mv2<N>(tab.K, a, tab.M, b, u);
#pragma unroll
    for (int r = 0; r < N; ++r) u[r] *= h;
    if (hang && hanging_line(m, 2, ta, tb, K)) interp<N, T, true>(tab.H, mask_sub(m, 2), u);
#pragma unroll
    for (int r = 0; r < N; ++r) B0[r * N2 + tb * N + ta] = u[r];
  }
  sync();
  // phase 6: x-lines (y = ta, z = tb): transposed x-interpolation
  if (block_hang) {
    if (active && hang && hanging_line(m, 0, ta, tb, K)) {
#pragma unroll
      for (int r = 0; r < N; ++r) u[r] = B0[tb * N2 + ta * N + r];
      interp<N, T, true>(tab.H, mask_sub(m, 0), u);
#pragma unroll
      for (int r = 0; r < N; ++r) B0[tb * N2 + ta * N + r] = u[r];
    }
    sync();
  }
  // phase 7: y-lines (x = ta, z = tb): transposed y-interpolation
  if (active) {
#pragma unroll
    for (int r = 0; r < N; ++r) u[r] = B0[tb * N2 + r * N + ta];
    if (hang && hanging_line(m, 1, ta, tb, K)) interp<N, T, true>(tab.H, mask_sub(m, 1), u);
  }
}

// The cell pipeline with even-odd 1D operators, z-sweeps first:
//   a = M_z u, b = K_z u;  c = M_y a, f = K_y a + M_y b;  out = h (K_x c + M_x f),
// which is h (K_x M_y M_z + M_x K_y M_z + M_x M_y K_z) u.  Input: this lane's
// z-line (x = ta, y = tb) of gathered values, so the z-sweeps start from
// registers.  In a wavefront without hanging nodes the result is this lane's
// x-line (y = ta, z = tb) and the function returns false.  Otherwise the
// interpolations of the hanging lines (they commute with each other) are
// applied around the sweeps: z in registers and y, x through LDS before,
// x in registers and y, z through LDS after; the result is then this lane's
// z-line (the gather layout) and the function returns true.  Hg (LDS) holds
// the interpolation matrices of both halves.  UNI: the wavefront holds one
// cell and m is wavefront-uniform (the interpolation then reads its matrices
// from the kernel arguments).  Must be called by all lanes of the wavefront.
template <int K, typename T, typename Sync, bool UNI = false>
__device__ __forceinline__ bool cell_pipeline_zfirst(T* __restrict__ B0, uint32_t m,
                                                     int any_hang, T h, const OpTab2<T, K + 1>& tab,
                                                     const T* __restrict__ Hg, int ta, int tb, T (&u)[K + 1]) {
  constexpr int N = K + 1, N2 = N * N;
  const Sync sync{};
  const bool hang = mask_hanging(m);
  if (any_hang) {
    if (hang && hanging_line(m, 2, ta, tb, K)) hang_interp<N, T, false, UNI>(Hg, mask_sub(m, 2), u);
#pragma unroll
    for (int c = 0; c < N; ++c) B0[c * N2 + tb * N + ta] = u[c];
    sync();
    if (hang && hanging_line(m, 1, ta, tb, K)) {
#pragma unroll
      for (int r = 0; r < N; ++r) u[r] = B0[tb * N2 + r * N + ta];
      hang_interp<N, T, false, UNI>(Hg, mask_sub(m, 1), u);
#pragma unroll
      for (int r = 0; r < N; ++r) B0[tb * N2 + r * N + ta] = u[r];
    }
    sync();
    if (hang && hanging_line(m, 0, ta, tb, K)) {
#pragma unroll
      for (int r = 0; r < N; ++r) u[r] = B0[tb * N2 + ta * N + r];
      hang_interp<N, T, false, UNI>(Hg, mask_sub(m, 0), u);
#pragma unroll
      for (int r = 0; r < N; ++r) B0[tb * N2 + ta * N + r] = u[r];
    }
    sync();
#pragma unroll
    for (int c = 0; c < N; ++c) u[c] = B0[c * N2 + tb * N + ta];  // own z-line, rewritten below
  }
  // One n^3 buffer per cell carries the four transposes one after the
  // other: a (z-lines -> y-lines), b (z -> y), c (y -> x), f (y -> x).  The
  // lanes of a cell are one wavefront, whose LDS operations execute in
  // order, so a buffer may be rewritten as soon as the previous read of it
  // has been issued; Sync keeps the compiler from reordering across.
  // Ordered to keep few values live: a dies into c and f once read back
  // along y, then b adds M_y b to f, and so on.
  T a[N], b[N], c[N], f[N];
  sym_mv<N>(tab.M, u, a);
  sym_mv<N>(tab.K, u, b);
#pragma unroll
  for (int q = 0; q < N; ++q) B0[q * N2 + tb * N + ta] = a[q];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) a[r] = B0[tb * N2 + r * N + ta];
  sym_mv<N>(tab.M, a, c);
  sym_mv<N>(tab.K, a, f);
  sync();
#pragma unroll
  for (int q = 0; q < N; ++q) B0[q * N2 + tb * N + ta] = b[q];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) a[r] = B0[tb * N2 + r * N + ta];
  sym_mv<N>(tab.M, a, b);
#pragma unroll
  for (int r = 0; r < N; ++r) f[r] += b[r];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) B0[tb * N2 + r * N + ta] = c[r];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) a[r] = B0[tb * N2 + ta * N + r];
  sym_mv<N>(tab.K, a, c);
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) B0[tb * N2 + r * N + ta] = f[r];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) a[r] = B0[tb * N2 + ta * N + r];
  sym_mv<N>(tab.M, a, b);
#pragma unroll
  for (int r = 0; r < N; ++r) u[r] = h * (c[r] + b[r]);
  if (!any_hang) return false;
  if (hang && hanging_line(m, 0, ta, tb, K)) hang_interp<N, T, true, UNI>(Hg, mask_sub(m, 0), u);
#pragma unroll
  for (int r = 0; r < N; ++r) B0[tb * N2 + ta * N + r] = u[r];  // this lane's own x-line
  sync();
  if (hang && hanging_line(m, 1, ta, tb, K)) {
#pragma unroll
    for (int r = 0; r < N; ++r) u[r] = B0[tb * N2 + r * N + ta];
    hang_interp<N, T, true, UNI>(Hg, mask_sub(m, 1), u);
#pragma unroll
    for (int r = 0; r < N; ++r) B0[tb * N2 + r * N + ta] = u[r];
  }
  sync();
#pragma unroll
  for (int c = 0; c < N; ++c) u[c] = B0[c * N2 + tb * N + ta];
  if (hang && hanging_line(m, 2, ta, tb, K)) hang_interp<N, T, true, UNI>(Hg, mask_sub(m, 2), u);
  return true;
}

// Per-lane constants of the operator kernel, for lane t = ta + n tb of a
// cell: entity slot and in-entity offsets (first node, first interior node,
// stride between interior nodes) of the lane's z-line (x = ta, y = tb) and
// x-line (y = ta, z = tb).  Built at compile time, read once per wavefront.
struct LaneLines {
  uint8_t zs0, zs1, zsm, zo0, zom, zst;
  uint8_t xs0, xs1, xsm, xo0, xom, xst;
};
template <int K>
struct LaneLineTable {
  LaneLines t[(K + 1) * (K + 1)];
};
template <int K>
constexpr LaneLineTable<K> make_lane_lines() {
  LaneLineTable<K> r{};
  for (int tb = 0; tb <= K; ++tb)
    for (int ta = 0; ta <= K; ++ta) {
      LaneLines& l = r.t[ta + (K + 1) * tb];
      l.zs0 = static_cast<uint8_t>(node_slot(ta, tb, 0, K));
      l.zs1 = static_cast<uint8_t>(node_slot(ta, tb, K, K));
      l.zsm = static_cast<uint8_t>(K > 1 ? node_slot(ta, tb, 1, K) : 26);
      l.zo0 = static_cast<uint8_t>(node_offset(ta, tb, 0, K));
      l.zom = static_cast<uint8_t>(K > 1 ? node_offset(ta, tb, 1, K) : 0);
      l.zst = static_cast<uint8_t>(K > 2 ? node_offset(ta, tb, 2, K) - node_offset(ta, tb, 1, K) : 0);
      l.xs0 = static_cast<uint8_t>(node_slot(0, ta, tb, K));
      l.xs1 = static_cast<uint8_t>(node_slot(K, ta, tb, K));
      l.xsm = static_cast<uint8_t>(K > 1 ? node_slot(1, ta, tb, K) : 26);
      l.xo0 = static_cast<uint8_t>(node_offset(0, ta, tb, K));
      l.xom = static_cast<uint8_t>(K > 1 ? node_offset(1, ta, tb, K) : 0);
      l.xst = static_cast<uint8_t>(K > 2 ? node_offset(2, ta, tb, K) - node_offset(1, ta, tb, K) : 0);
    }
  return r;
}
template <int K>
__constant__ LaneLineTable<K> kLaneLines = make_lane_lines<K>();

// Gauss-point tables of the operator on mapped cells: S[q][i] = l_i(g_q)
// (Gauss-Lobatto basis at the Gauss points), D[q][p] = L_p'(g_q) (derivative
// of the Lagrange basis on the Gauss points: gradients from point values),
// the Gauss points g and weights w on [0, 1].
template <typename T, int N>
struct MapTab {
  T S[N * N];
  T D[N * N];
  T g[N];
  T w[N];
};

template <typename T, int N>
MapTab<T, N> make_maptab() {
  const Tables1D& t = tables(N - 1);
  MapTab<T, N> m;
  for (int q = 0; q < N; ++q) {
    m.g[q] = static_cast<T>(t.qp[q]);
    m.w[q] = static_cast<T>(t.qw[q]);
    for (int i = 0; i < N; ++i) {
      m.S[q * N + i] = static_cast<T>(t.S[q * N + i]);
      m.D[q * N + i] = static_cast<T>(lagrange_deriv(t.qp, i, t.qp[q]));
    }
  }
  return m;
}

// y = A x (TRANS: y = A^T x) for an n x n table A
template <int N, typename T, bool TRANS>
__device__ __forceinline__ void mat_mv(const T* __restrict__ A, const T (&x)[N], T (&y)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T acc = (TRANS ? A[i] : A[i * N]) * x[0];
#pragma unroll
    for (int j = 1; j < N; ++j) acc += (TRANS ? A[j * N + i] : A[i * N + j]) * x[j];
    y[i] = acc;
  }
}

// Geometry of one cell of a mapped level: the coarse cell's map coefficients
// (monomial form, see geometry.hpp) and the cell's box inside it,
// t = (r + xi) * scale.
template <typename T>
struct CellGeo {
  const T* A;
  T r[3];
  T scale;
};

// The cell pipeline C^T S^T Q S C on a mapped cell (Eq. impl:mf with the
// general Q_e): values at the Gauss points by three sweeps of S, reference
// gradients at the points by sweeps of D, the metric term
// c_e w_q |det J| J^{-1} J^{-T} at every point (J from the cell's trilinear
// map), the transposed sweeps D^T and S^T.  The one n^3 buffer B of the cell
// re-distributes the values between the line directions.  Input: this lane's
// z-line (x = ta, y = tb) of gathered slot values; output: the same z-line
// of the result (the gather layout).  Hanging lines are interpolated as in
// the axis-aligned pipeline (before: z in registers, y and x in LDS; after:
// the transposes, z in registers, y and x in LDS).  Must be called by all
// lanes of the wavefront.
template <int K, typename T, typename Sync>
__device__ __forceinline__ void cell_pipeline_mapped(T* __restrict__ B, uint32_t m, int any_hang, T coef,
                                                     const MapTab<T, K + 1>& mt, const CellGeo<T>& geo,
                                                     const T* __restrict__ Hg, int ta, int tb, T (&u)[K + 1]) {
  constexpr int N = K + 1, N2 = N * N;
  const Sync sync{};
  const bool hang = mask_hanging(m);
  auto zl = [&](int c) { return c * N2 + tb * N + ta; };  // z-line (x = ta, y = tb)
  auto yl = [&](int r) { return tb * N2 + r * N + ta; };  // y-line (x = ta, z = tb)
  auto xl = [&](int r) { return tb * N2 + ta * N + r; };  // x-line (y = ta, z = tb)
  if (any_hang) {
    if (hang && hanging_line(m, 2, ta, tb, K)) interp_lds<N, T, false>(Hg, mask_sub(m, 2), u);
#pragma unroll
    for (int c = 0; c < N; ++c) B[zl(c)] = u[c];
    sync();
    if (hang && hanging_line(m, 1, ta, tb, K)) {
#pragma unroll
      for (int r = 0; r < N; ++r) u[r] = B[yl(r)];
      interp_lds<N, T, false>(Hg, mask_sub(m, 1), u);
#pragma unroll
      for (int r = 0; r < N; ++r) B[yl(r)] = u[r];
    }
    sync();
    if (hang && hanging_line(m, 0, ta, tb, K)) {
#pragma unroll
      for (int r = 0; r < N; ++r) u[r] = B[xl(r)];
      interp_lds<N, T, false>(Hg, mask_sub(m, 0), u);
#pragma unroll
      for (int r = 0; r < N; ++r) B[xl(r)] = u[r];
    }
    sync();
#pragma unroll
    for (int c = 0; c < N; ++c) u[c] = B[zl(c)];
    sync();
  }
  T v[N], w[N], gx[N], gy[N], gz[N];
  // values at the Gauss points: z, y, x
  mat_mv<N, T, false>(mt.S, u, v);
#pragma unroll
  for (int c = 0; c < N; ++c) B[zl(c)] = v[c];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) w[r] = B[yl(r)];
  mat_mv<N, T, false>(mt.S, w, v);
#pragma unroll
  for (int r = 0; r < N; ++r) B[yl(r)] = v[r];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) w[r] = B[xl(r)];
  mat_mv<N, T, false>(mt.S, w, v);
  mat_mv<N, T, false>(mt.D, v, gx);  // d/dxi_1 along this x-line
#pragma unroll
  for (int r = 0; r < N; ++r) B[xl(r)] = v[r];
  sync();
  // d/dxi_2 (y-lines) and d/dxi_3 (z-lines), brought to this lane's x-line
#pragma unroll
  for (int r = 0; r < N; ++r) w[r] = B[yl(r)];
#pragma unroll
  for (int r = 0; r < N; ++r) v[r] = B[zl(r)];
  mat_mv<N, T, false>(mt.D, w, gy);
  mat_mv<N, T, false>(mt.D, v, gz);
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) B[yl(r)] = gy[r];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) gy[r] = B[xl(r)];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) B[zl(r)] = gz[r];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) gz[r] = B[xl(r)];
  // quadrature points (x = r, y = ta, z = tb): flux G grad u
  {
    const T t2 = (geo.r[1] + mt.g[ta]) * geo.scale, t3 = (geo.r[2] + mt.g[tb]) * geo.scale;
    const T wyz = mt.w[ta] * mt.w[tb] * coef;
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const T t1 = (geo.r[0] + mt.g[r]) * geo.scale;
      T J[3][3];
      geo_jacobian<T>(geo.A, t1, t2, t3, J);
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int e = 0; e < 3; ++e) J[d][e] *= geo.scale;
      T G[6];
      geo_metric<T>(J, wyz * mt.w[r], G);
      const T a = gx[r], b = gy[r], c = gz[r];
      gx[r] = G[0] * a + G[1] * b + G[2] * c;
      gy[r] = G[1] * a + G[3] * b + G[4] * c;
      gz[r] = G[2] * a + G[4] * b + G[5] * c;
    }
  }
  // transposed gradient sweeps, summed along this lane's x-line
  mat_mv<N, T, true>(mt.D, gx, v);
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) B[xl(r)] = gy[r];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) w[r] = B[yl(r)];
  mat_mv<N, T, true>(mt.D, w, gy);
#pragma unroll
  for (int r = 0; r < N; ++r) B[yl(r)] = gy[r];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) v[r] += B[xl(r)];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) B[xl(r)] = gz[r];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) w[r] = B[zl(r)];
  mat_mv<N, T, true>(mt.D, w, gz);
#pragma unroll
  for (int r = 0; r < N; ++r) B[zl(r)] = gz[r];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) v[r] += B[xl(r)];
  // back to the nodes: S^T along x, y, z
  mat_mv<N, T, true>(mt.S, v, w);
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) B[xl(r)] = w[r];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) v[r] = B[yl(r)];
  mat_mv<N, T, true>(mt.S, v, w);
#pragma unroll
  for (int r = 0; r < N; ++r) B[yl(r)] = w[r];
  sync();
#pragma unroll
  for (int r = 0; r < N; ++r) v[r] = B[zl(r)];
  mat_mv<N, T, true>(mt.S, v, u);
  if (!any_hang) return;
  if (hang && hanging_line(m, 2, ta, tb, K)) interp_lds<N, T, true>(Hg, mask_sub(m, 2), u);
  sync();
#pragma unroll
  for (int c = 0; c < N; ++c) B[zl(c)] = u[c];
  sync();
  if (hang && hanging_line(m, 1, ta, tb, K)) {
#pragma unroll
    for (int r = 0; r < N; ++r) w[r] = B[yl(r)];
    interp_lds<N, T, true>(Hg, mask_sub(m, 1), w);
#pragma unroll
    for (int r = 0; r < N; ++r) B[yl(r)] = w[r];
  }
  sync();
  if (hang && hanging_line(m, 0, ta, tb, K)) {
#pragma unroll
    for (int r = 0; r < N; ++r) w[r] = B[xl(r)];
    interp_lds<N, T, true>(Hg, mask_sub(m, 0), w);
#pragma unroll
    for (int r = 0; r < N; ++r) B[xl(r)] = w[r];
  }
  sync();
#pragma unroll
  for (int c = 0; c < N; ++c) u[c] = B[zl(c)];
}

// geometry of cell `cell` of a mapped level (its lattice position ijk and
// level l; the coarse grid has n0 cells per axis)
template <typename T>
__device__ __forceinline__ CellGeo<T> cell_geo(const T* __restrict__ table, const int32_t* __restrict__ ijk,
                                               int64_t cell, int l, int n0) {
  CellGeo<T> g;
  const int i = ijk[3 * cell], j = ijk[3 * cell + 1], k = ijk[3 * cell + 2];
  const int I = i >> l, J = j >> l, Kc = k >> l;
  g.A = table + (static_cast<int64_t>(I) + n0 * (J + static_cast<int64_t>(n0) * Kc)) * 24;
  g.r[0] = static_cast<T>(i - (I << l));
  g.r[1] = static_cast<T>(j - (J << l));
  g.r[2] = static_cast<T>(k - (Kc << l));
  g.scale = static_cast<T>(ldexp(1.0, -l));
  return g;
}

// Shared-DoF route of the batch kernel, or-ed into the fused kind by the
// launcher: the shared DoFs' sums are added with global atomics (into dst for
// the plain operator, else into an accumulator that finish_shared_kernel
// completes) instead of being written as partial sums
constexpr int FUSE_ATOMIC = 4;
constexpr int base_kind(int fk) { return fk & 3; }

// Final value t = (A x) of DoF g, vector v, and the fused step applied to it
template <typename S, typename T, int FK>
__device__ __forceinline__ void finish_dof(const FusedStep& f, int64_t g, int nv, int v, T t, T* __restrict__ dst) {
  const int64_t e = g * nv + v;
  if constexpr (base_kind(FK) == FUSE_NONE) {
    dst[e] = t;
  } else if constexpr (base_kind(FK) == FUSE_RESIDUAL) {
    static_cast<S*>(f.r)[e] = store_as<S>(load_as<T>(static_cast<const S*>(f.b)[e]) - t);
  } else {
    S* d = static_cast<S*>(f.d);
    S* x = static_cast<S*>(f.x);
    const T di = static_cast<const T*>(f.dinv)[g];
    const T dd = f.c_dd != 0.0 ? static_cast<T>(f.c_dd) * load_as<T>(d[e]) : T(0);
    const T dn = dd + static_cast<T>(f.c_r) * di * (load_as<T>(static_cast<const S*>(f.b)[e]) - t);
    x[e] = store_as<S>(load_as<T>(x[e]) + dn);
    d[e] = store_as<S>(dn);
  }
}

// Operator evaluation by cell batches.  The blocks are persistent: the
// batches are split into 8 contiguous ranges, one per XCD (block i runs on XCD
// i mod 8), and the blocks of an XCD take the batches of its range in turn,
// so neighbouring batches share that XCD's L2.  Per batch, the batch's DoFs
// are loaded into LDS (shared DoFs through their index list, exclusive DoFs as
// one contiguous range), the cells are evaluated group by group from LDS and
// their contributions accumulated in LDS, then the exclusive DoFs are stored
// contiguously and the shared DoFs either added with global atomics
// (FUSE_ATOMIC route, one vector: into dst, or into the accumulator in the
// partial buffer when a step is fused; either cleared before) or written as
// this batch's partial sums (reduced afterwards).  gridDim.x is a multiple
// of 8.
// register budget: 4 wavefronts per SIMD (two blocks per CU, as the LDS
// allows); the operator of mapped cells, which holds three gradient
// components and the metric terms of a line of points, gets the registers of
// 2 wavefronts per SIMD instead of spilling
template <int K, int FK, int GEO>
struct BatchWavesPerEu {
  static constexpr int value = GEO ? 2 : 4;
};

template <int K, typename S, typename T, int FK, int GEO, bool DET>
__global__ void __launch_bounds__(BATCH_WAVES * 64)
    __attribute__((amdgpu_waves_per_eu(BatchWavesPerEu<K, FK, GEO>::value)))
    vmult_batch_kernel(const CellMeta* __restrict__ meta, const int32_t* __restrict__ bcell,
                       const int32_t* __restrict__ bsh, const int32_t* __restrict__ bex,
                       const int32_t* __restrict__ sh_idx, int64_t nb,
                       int64_t n_shared, double h0, OpTab2<T, K + 1> tab, const S* __restrict__ src,
                       T* __restrict__ partial, T* __restrict__ dst, int nv, FusedStep fs,
                       const T* __restrict__ geo, const int32_t* __restrict__ ijk, int n0, MapTab<T, K + 1> mt) {
  constexpr int N = K + 1, N2 = N * N, N3 = N2 * N, CPW = cells_per_wave(N), MCAP = batch_mcap(K);
  constexpr int NZ = batch_zero_entries(K), ZB = MCAP;  // zero block behind the batch's DoFs
  constexpr int BT = BATCH_WAVES * 64, PER = (MCAP + BT - 1) / BT;
  __shared__ T in_[MCAP + NZ];
  __shared__ double out_[MCAP + NZ];  // contributions accumulate in FP64 (also for FP32 arithmetic)
  __shared__ T Hg[2 * N2];
  constexpr bool META_LDS = batch_meta_in_lds(K);
  __shared__ CellMeta metaL[META_LDS ? batch_max_cells(K) : 1];
  __shared__ T buf0[(BATCH_WAVES * CPW + 1) * N3];
  for (int i = threadIdx.x; i < NZ; i += BT) in_[ZB + i] = T(0);
  for (int i = threadIdx.x; i < 2 * N2; i += BT) Hg[i] = tab.Hg[i];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int lc = lane / N2;
  const int t = lane - lc * N2;
  const bool lane_used = lc < CPW;
  const int ta = t % N, tb = t / N;
  // lanes without a cell work on the block's spare buffers (results unused)
  T* B0 = buf0 + (lane_used ? wave * CPW + lc : BATCH_WAVES * CPW) * N3;
  const LaneLines ll = kLaneLines<K>.t[t];
  const int gsm = ll.zsm, go0 = ll.zo0, gom = ll.zom, gst = ll.zst;
  const int ssm = ll.xsm, so0 = ll.xo0, som = ll.xom, sst = ll.xst;
  // the six slots of the lane's z-line and x-line (each < 27), five bits
  // apiece: the metadata fetch unpacks them each time instead of holding six
  // 64-bit offsets through the batch loop
  const uint32_t slots = ll.zs0 | (ll.zs1 << 5) | (ll.zsm << 10) | (ll.xs0 << 15) | (ll.xs1 << 20) |
                         (static_cast<uint32_t>(ll.xsm) << 25);
  struct Pre {
    int g0, g1, gm, s0, s1, sm;
    uint32_t mask;
  };

  if constexpr ((FK & FUSE_ATOMIC) != 0) nv = 1;  // (one vector: the index arithmetic folds)
  const int64_t per = (nb + 7) / 8;
  const int64_t lo = (blockIdx.x % 8) * per;
  const int64_t hi = lo + per < nb ? lo + per : nb;
  // several interleaved vectors: nv blocks of one XCD (consecutive block
  // indices there) take the same batch at the same time, one vector each,
  // so that the nv values of a DoF, adjacent in memory, are read once into
  // that XCD's L2 and their partial-line writes meet there.  (Vectors one
  // after the other in one block left a whole pass of the other blocks'
  // traffic between two passes over a line, so that it was fetched and
  // written back up to nv times.)  The launch gives every XCD at least nv
  // blocks.
  const int groups = static_cast<int>(gridDim.x / 8) / nv;
  const int j = static_cast<int>(blockIdx.x / 8);
  if (j >= groups * nv) return;  // (whole block: no barrier passed yet)
  const int v = j % nv;
  const int64_t b0 = lo + j / nv;
  for (int64_t w = 0;; ++w) {
    const int64_t b = b0 + w * groups;
    if (b >= hi) break;
    const int c0 = bcell[b], c1 = bcell[b + 1];
    const int sh0 = bsh[b], nsh = bsh[b + 1] - sh0;
    const int64_t ex0 = n_shared + bex[b];
    const int m = nsh + (bex[b + 1] - bex[b]);
    // stage the batch's DoFs: all index loads of a thread, then all value
    // loads, then the LDS stores, so that the loads of a thread overlap
    {
      int32_t gi[PER];  // DoF indices (a level has fewer than 2^31 DoFs)
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int i = threadIdx.x + q * BT;
        gi[q] = i < nsh ? sh_idx[sh0 + i] : static_cast<int32_t>(ex0 + (i - nsh));
      }
      T val[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int i = threadIdx.x + q * BT;
        val[q] = i < m ? load_as<T>(src[static_cast<int64_t>(gi[q]) * nv + v]) : T(0);
      }
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int i = threadIdx.x + q * BT;
        if (i < m) {
          in_[i] = val[q];
          out_[i] = 0.0;
        }
      }
    }
    // metadata of this lane's cell, fetched one cell group ahead: the six
    // local entity starts of its z-line and x-line and the mask (the loads are
    // unconditional, from the batch's first cell for lanes without a cell, so
    // that the wait for them can be counted exactly; such lanes then point at
    // the zero block)
    if constexpr (META_LDS) {  // the batch's cell records, 16 bytes per thread
      const uint4* gsrc = reinterpret_cast<const uint4*>(meta + c0);
      uint4* ldst = reinterpret_cast<uint4*>(metaL);
      for (int i = threadIdx.x; i < (c1 - c0) * 4; i += BT) ldst[i] = gsrc[i];
    }
    auto fetch = [&](int64_t cell) {
      const bool ok = lane_used && cell < c1;
      const CellMeta* M = META_LDS ? metaL + (ok ? cell - c0 : 0) : meta + (ok ? cell : c0);
      const uint16_t* L = M->loc;
      uint32_t sl = slots;
      asm volatile("" : "+v"(sl));  // (keeps the unpacking here, not hoisted out of the loops)
      Pre p{L[sl & 31u],         L[(sl >> 5) & 31u],  L[(sl >> 10) & 31u],
            L[(sl >> 15) & 31u], L[(sl >> 20) & 31u], L[sl >> 25],         M->mask};
      p.g0 = ok ? p.g0 : ZB;
      p.g1 = ok ? p.g1 : ZB;
      p.gm = ok ? p.gm : ZB;
      p.s0 = ok ? p.s0 : ZB;
      p.s1 = ok ? p.s1 : ZB;
      p.sm = ok ? p.sm : ZB;
      p.mask = ok ? p.mask : 0u;
      return p;
    };
    int cw = c0 + wave * CPW;
    if constexpr (META_LDS) __syncthreads();
    Pre nx = fetch(cw + lc);
    if constexpr (!META_LDS) __syncthreads();
    // deterministic mode: every wavefront runs the same number of rounds (the
    // last one partly without cells), and the scatter below goes one cell at
    // a time in cell order
    const int rounds = DET ? (c1 - c0 + BATCH_WAVES * CPW - 1) / (BATCH_WAVES * CPW) : 0;
    for (int round = 0;; ++round, cw += BATCH_WAVES * CPW) {
      if constexpr (DET) {
        if (round >= rounds) break;
      } else {
        if (cw >= c1) break;
      }
      const Pre cur = nx;
      nx = fetch(cw + BATCH_WAVES * CPW + lc);
      // one cell per wavefront: its mask is uniform (lanes without a cell
      // take it too; their results are discarded)
      constexpr bool UNI = CPW == 1 && GEO == 0;
      const uint32_t mk = UNI ? __builtin_amdgcn_readfirstlane(cur.mask) : cur.mask;
      const int wave_hang = UNI ? (mask_hanging(mk) ? 1 : 0) : __any(mask_hanging(mk) ? 1 : 0);
      const T h = static_cast<T>(ldexp(h0, -mask_level(mk)) * static_cast<double>(mask_coef(mk)));
      T u[N];
      u[0] = in_[cur.g0 + go0];
      u[K] = in_[cur.g1 + go0];
      if constexpr (K > 1) {
#pragma unroll
        for (int c = 1; c < K; ++c) u[c] = in_[cur.gm + gom + (c - 1) * gst];
      }
      bool zline = true;
      if constexpr (GEO != 0) {  // mapped cell: its own map from its coarse cell
        const int64_t cell = (lane_used && cw + lc < c1) ? cw + lc : c0;
        const CellGeo<T> g = cell_geo<T>(geo, ijk, cell, mask_level(mk), n0);
        cell_pipeline_mapped<K, T, WaveSync>(B0, mk, wave_hang, static_cast<T>(mask_coef(mk)), mt, g, Hg, ta, tb, u);
      } else {
        zline = cell_pipeline_zfirst<K, T, WaveSync, UNI>(B0, mk, wave_hang, h, tab, Hg, ta, tb, u);
      }
      // scatter-add along the result line, skipping absent entities and
      // lanes without a cell (they point at the zero block); a line through
      // the cell interior (slot 26) holds DoFs of this cell only
      const int s0 = zline ? cur.g0 : cur.s0, s1 = zline ? cur.g1 : cur.s1, sm = zline ? cur.gm : cur.sm;
      const int o0 = zline ? go0 : so0, om = zline ? gom : som, st = zline ? gst : sst;
      auto add = [&](int i, T v) {
        if constexpr (DET) out_[i] += static_cast<double>(v);  // the only writer at this moment
        else atomicAdd(&out_[i], static_cast<double>(v));
      };
      auto scatter = [&]() {
        if (s0 < ZB) add(s0 + o0, u[0]);
        if (s1 < ZB) add(s1 + o0, u[K]);
        if constexpr (K > 1) {
          if (sm < ZB) {
            if ((zline ? gsm : ssm) == 26) {
#pragma unroll
              for (int r = 1; r < K; ++r) out_[sm + om + (r - 1) * st] = static_cast<double>(u[r]);
            } else {
#pragma unroll
              for (int r = 1; r < K; ++r) add(sm + om + (r - 1) * st, u[r]);
            }
          }
        }
      };
      if constexpr (DET) {
        for (int q = 0; q < BATCH_WAVES * CPW; ++q) {  // cell c0 + round * (block's cells) + q
          if (lane_used && wave * CPW + lc == q) scatter();
          __syncthreads();
        }
      } else {
        scatter();
      }
      WaveSync{}();  // the next cell group reuses this wavefront's buffers
    }
    // write back: the shared DoFs' sums atomically into dst or the
    // accumulator (their indices read again: keeping them in registers
    // through the evaluation would spill) or as one contiguous range of
    // partial sums (the batch's part of the partial buffer); exclusive DoFs
    // in place, with the fused step
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = threadIdx.x + q * BT;
      if (i < nsh) {
        if constexpr ((FK & FUSE_ATOMIC) != 0)
          unsafeAtomicAdd(&(base_kind(FK) == FUSE_NONE ? dst : partial)[sh_idx[sh0 + i]], static_cast<T>(out_[i]));
        else partial[static_cast<int64_t>(sh0 + i) * nv + v] = static_cast<T>(out_[i]);
      } else if (i < m) finish_dof<S, T, FK>(fs, ex0 + (i - nsh), nv, v, static_cast<T>(out_[i]), dst);
    }
    __syncthreads();  // the next batch or vector overwrites in_ and out_
  }
}

template <typename T>
__global__ void clear_shared_kernel(int64_t n, T* __restrict__ dst) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[i] = T(0);
}

// the fused step on the shared DoFs of one vector, from their sums (A x)_s
// accumulated atomically in acc
template <typename S, typename T, int FK>
__global__ void finish_shared_kernel(int64_t n_shared, const T* __restrict__ acc, T* __restrict__ dst, FusedStep fs) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n_shared;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    finish_dof<S, T, FK>(fs, i, 1, 0, acc[i], dst);
}

// (A x)_s = sum of the partial sums of shared DoF s, in the fixed order of its
// batches (red_idx holds their positions in the batch-ordered partial
// buffer), then the fused step
template <typename S, typename T, int FK>
__global__ void reduce_shared_kernel(int64_t n_shared, int nv, const int32_t* __restrict__ red_off,
                                     const int32_t* __restrict__ red_idx, const T* __restrict__ partial,
                                     T* __restrict__ dst, FusedStep fs) {
  const int64_t n = n_shared * nv;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t sd = i / nv;
    const int v = static_cast<int>(i - sd * nv);
    T acc = T(0);
    for (int j = red_off[sd]; j < red_off[sd + 1]; ++j)
      acc += partial[static_cast<int64_t>(red_idx[j]) * nv + v];
    finish_dof<S, T, FK>(fs, sd, nv, v, acc, dst);
  }
}

// The same for NV interleaved vectors, one thread per shared DoF: the NV
// values of a partial sum are one aligned vector load, its index is read once
// for all of them, and every value is summed in the same order as above
template <typename S, typename T, int FK, int NV>
__global__ void reduce_shared_vec_kernel(int64_t n_shared, const int32_t* __restrict__ red_off,
                                         const int32_t* __restrict__ red_idx, const T* __restrict__ partial,
                                         T* __restrict__ dst, FusedStep fs) {
  typedef T VecT __attribute__((ext_vector_type(NV)));
  for (int64_t sd = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; sd < n_shared;
       sd += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    VecT acc = T(0);
    for (int j = red_off[sd]; j < red_off[sd + 1]; ++j)
      acc += *reinterpret_cast<const VecT*>(partial + static_cast<int64_t>(red_idx[j]) * NV);
#pragma unroll
    for (int v = 0; v < NV; ++v) finish_dof<S, T, FK>(fs, sd, NV, v, acc[v], dst);
  }
}

// Does the hanging-node interpolation C_e touch node (a, b, c)?  Only if one
// of the three lines through the node is interpolated: otherwise C_e e_s =
// e_s for its slot s (the in-place line interpolations mix values along
// their own lines only), and (C_e^T A_e C_e)_ss = A_e(s, s).
__device__ __forceinline__ bool node_constrained(uint32_t m, int a, int b, int c, int k) {
  return hanging_line(m, 0, b, c, k) || hanging_line(m, 1, a, c, k) || hanging_line(m, 2, a, b, k);
}

// Diagonal (Eq. impl:mf:diagonal).  d_e(i) = A_e(i,i) = h (K_aa M_bb M_cc +
// M_aa K_bb M_cc + M_aa M_bb K_cc) for every node that the cell's hanging-node
// interpolation leaves alone; for the others (the nodes of hanging faces and
// edges) apply C_e^T A_e C_e to the unit slot vector e_s and keep entry s.
// One cell per block, n^2 threads.
template <int K>
__global__ void __launch_bounds__((K + 1) * (K + 1))
    diag_kernel(const int32_t* __restrict__ ent, const uint32_t* __restrict__ mask, int64_t nc, double h0,
                OpTab<double, K + 1> tab, double* __restrict__ diag, const int32_t* __restrict__ cells) {
  constexpr int N = K + 1, N2 = N * N, N3 = N2 * N;
  __shared__ double B0[N3];
  __shared__ double B1[N3];
  const int64_t cell = cells ? cells[blockIdx.x] : blockIdx.x;  // cells: one colour (deterministic mode)
  const int ta = threadIdx.x % N, tb = threadIdx.x / N;
  const uint32_t m = mask[cell];
  const double h = ldexp(h0, -mask_level(m)) * static_cast<double>(mask_coef(m));
  double d[N];  // y-line (x = ta, z = tb)
#pragma unroll
  for (int r = 0; r < N; ++r)
    d[r] = h * (tab.K[ta * N + ta] * tab.M[r * N + r] * tab.M[tb * N + tb] +
                tab.M[ta * N + ta] * tab.K[r * N + r] * tab.M[tb * N + tb] +
                tab.M[ta * N + ta] * tab.M[r * N + r] * tab.K[tb * N + tb]);
  if (mask_hanging(m)) {
    for (int s = 0; s < N3; ++s) {
      const int sa = s % N, sb = (s / N) % N, sc = s / N2;
      if (!node_constrained(m, sa, sb, sc, K)) continue;  // uniform over the block
      double u[N];
#pragma unroll
      for (int c = 0; c < N; ++c) u[c] = (ta == sa && tb == sb && c == sc) ? 1.0 : 0.0;
      cell_pipeline<K, double, WaveSync>(B0, B1, true, m, 1, h, tab, ta, tb, u);
      if (ta == sa && tb == sc) {
#pragma unroll
        for (int r = 0; r < N; ++r)
          if (r == sb) d[r] = u[r];
      }
      WaveSync{}();
    }
  }
  scatter_yline<K>(ent, nc, cell, ta, tb, d, diag, 1, 0, cells != nullptr);
}

// scatter-add of the line of nodes (a, b, 0..k) (along z), as scatter_yline
template <int K, typename T, bool INTERIOR = true>
__device__ __forceinline__ void scatter_zline(const int32_t* __restrict__ ent, int64_t nc, int64_t cell, int a,
                                              int b, const T (&w)[K + 1], T* __restrict__ dst, bool plain = false) {
  const int s0 = node_slot(a, b, 0, K), s1 = node_slot(a, b, K, K);
  const int o0 = node_offset(a, b, 0, K);
  const int32_t e0 = ent[s0 * nc + cell], e1 = ent[s1 * nc + cell];
  if (e0 >= 0) scatter_add(&dst[e0 + o0], w[0], plain);
  if (e1 >= 0) scatter_add(&dst[e1 + o0], w[K], plain);
  if constexpr (K > 1) {
    const int sm = node_slot(a, b, 1, K);
    const int om = node_offset(a, b, 1, K);
    const int st = K > 2 ? node_offset(a, b, 2, K) - om : 0;
    const int32_t em = ent[sm * nc + cell];
    if (em >= 0 && (INTERIOR || sm != 26)) {
#pragma unroll
      for (int c = 1; c < K; ++c) {
        if (sm == 26) dst[em + om + (c - 1) * st] = w[c];
        else scatter_add(&dst[em + om + (c - 1) * st], w[c], plain);
      }
    }
  }
}

// Diagonal of a mapped cell without constraints, A_e(i,i) =
// sum_q grad phi_i(q)^T G_q grad phi_i(q), G_q = c_e w_q |det J| J^-1 J^-T:
// with phi_i = l_a l_b l_c, d_xi1 phi_i = l'_a l_b l_c etc., every product of
// two gradient components is a product of 1D factors, so the six symmetric
// components of G contract with squared 1D tables (E = S.S, F = S'.S',
// X = S'.S elementwise; S' = l'(g_q)) axis by axis: 6 x 3 sweeps.  One cell
// per block of n^2 threads.  In cells with hanging nodes the nodes that the
// interpolation touches are left to diag_mapped_kernel (written as 0 here).
template <typename T, int N>
struct DiagTab {
  T E[N * N], F[N * N], X[N * N];  // [q][a]
};

template <int K>
__global__ void __launch_bounds__((K + 1) * (K + 1))
    diag_mapped_direct_kernel(const int32_t* __restrict__ ent, const uint32_t* __restrict__ mask, int64_t nc,
                              const double* __restrict__ geo, const int32_t* __restrict__ ijk, int n0,
                              MapTab<double, K + 1> mt, DiagTab<double, K + 1> dt, double* __restrict__ diag,
                              const int32_t* __restrict__ cells) {
  constexpr int N = K + 1, N2 = N * N, N3 = N2 * N;
  __shared__ double B[N3];
  const int64_t cell = cells ? cells[blockIdx.x] : blockIdx.x;
  const uint32_t m = mask[cell];
  const int ta = threadIdx.x % N, tb = threadIdx.x / N;
  const CellGeo<double> g = cell_geo<double>(geo, ijk, cell, mask_level(m), n0);
  const double coef = static_cast<double>(mask_coef(m));
  double G[6][N];  // this lane's x-line of quadrature points (x = r, y = ta, z = tb)
  {
    const double t2 = (g.r[1] + mt.g[ta]) * g.scale, t3 = (g.r[2] + mt.g[tb]) * g.scale;
#pragma unroll
    for (int r = 0; r < N; ++r) {
      double J[3][3], Gq[6];
      geo_jacobian<double>(g.A, (g.r[0] + mt.g[r]) * g.scale, t2, t3, J);
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int e = 0; e < 3; ++e) J[d][e] *= g.scale;
      geo_metric<double>(J, coef * mt.w[r] * mt.w[ta] * mt.w[tb], Gq);
#pragma unroll
      for (int q = 0; q < 6; ++q) G[q][r] = Gq[q];
    }
  }
  // (component of G, factor, x table, y table, z table): g00 F E E, g11 E F E,
  // g22 E E F, 2 g01 X X E, 2 g02 X E X, 2 g12 E X X
  const double* tabs[6][3] = {{dt.F, dt.E, dt.E}, {dt.X, dt.X, dt.E}, {dt.X, dt.E, dt.X},
                              {dt.E, dt.F, dt.E}, {dt.E, dt.X, dt.X}, {dt.E, dt.E, dt.F}};
  const double fac[6] = {1.0, 2.0, 2.0, 1.0, 2.0, 1.0};
  double d[N];
#pragma unroll
  for (int c = 0; c < N; ++c) d[c] = 0.0;
  for (int q = 0; q < 6; ++q) {
    double v[N], w[N];
#pragma unroll
    for (int r = 0; r < N; ++r) v[r] = fac[q] * G[q][r];
    mat_mv<N, double, true>(tabs[q][0], v, w);  // x: node a <- point
    WaveSync{}();
#pragma unroll
    for (int r = 0; r < N; ++r) B[tb * N2 + ta * N + r] = w[r];
    WaveSync{}();
#pragma unroll
    for (int r = 0; r < N; ++r) v[r] = B[tb * N2 + r * N + ta];
    mat_mv<N, double, true>(tabs[q][1], v, w);  // y
#pragma unroll
    for (int r = 0; r < N; ++r) B[tb * N2 + r * N + ta] = w[r];
    WaveSync{}();
#pragma unroll
    for (int r = 0; r < N; ++r) v[r] = B[r * N2 + tb * N + ta];
    mat_mv<N, double, true>(tabs[q][2], v, w);  // z
#pragma unroll
    for (int c = 0; c < N; ++c) d[c] += w[c];
  }
  if (mask_hanging(m)) {
#pragma unroll
    for (int c = 0; c < N; ++c)
      if (node_constrained(m, ta, tb, c, K)) d[c] = 0.0;
  }
  scatter_zline<K>(ent, nc, cell, ta, tb, d, diag, cells != nullptr);
}

// Diagonal of a mapped cell with hanging nodes (Eq. impl:mf:diagonal), the
// nodes that the interpolation touches: the cell operator C_e^T A_e C_e
// applied to the unit slot vector e_s, entry s kept (the other nodes come
// from diag_mapped_direct_kernel; the cell interior is never touched and not
// written here).  One cell per block of n^2 threads (one wavefront).
template <int K>
__global__ void __launch_bounds__((K + 1) * (K + 1))
    diag_mapped_kernel(const int32_t* __restrict__ ent, const uint32_t* __restrict__ mask, int64_t nc,
                       const double* __restrict__ geo, const int32_t* __restrict__ ijk, int n0,
                       MapTab<double, K + 1> mt, OpTab2<double, K + 1> tab, double* __restrict__ diag,
                       const int32_t* __restrict__ cells) {
  constexpr int N = K + 1, N2 = N * N, N3 = N2 * N;
  __shared__ double B[N3];
  __shared__ double Hg[2 * N2];
  for (int i = threadIdx.x; i < 2 * N2; i += blockDim.x) Hg[i] = tab.Hg[i];
  __syncthreads();
  const int64_t cell = cells ? cells[blockIdx.x] : blockIdx.x;
  const int ta = threadIdx.x % N, tb = threadIdx.x / N;
  const uint32_t m = mask[cell];
  if (!mask_hanging(m)) return;  // (diag_mapped_direct_kernel)
  const CellGeo<double> g = cell_geo<double>(geo, ijk, cell, mask_level(m), n0);
  const double coef = static_cast<double>(mask_coef(m));
  const int any_hang = 1;
  double d[N];
#pragma unroll
  for (int c = 0; c < N; ++c) d[c] = 0.0;
  for (int sc = 0; sc < N; ++sc)
    for (int sb = 0; sb < N; ++sb)
      for (int sa = 0; sa < N; ++sa) {
        if (!node_constrained(m, sa, sb, sc, K)) continue;  // uniform over the block
        double u[N];
#pragma unroll
        for (int c = 0; c < N; ++c) u[c] = (ta == sa && tb == sb && c == sc) ? 1.0 : 0.0;
        cell_pipeline_mapped<K, double, WaveSync>(B, m, any_hang, coef, mt, g, Hg, ta, tb, u);
        if (ta == sa && tb == sb) {
#pragma unroll
          for (int c = 0; c < N; ++c)
            if (c == sc) d[c] += u[c];
        }
        WaveSync{}();
      }
  scatter_zline<K, double, false>(ent, nc, cell, ta, tb, d, diag, cells != nullptr);
}

// Constraint distribution: gather G_e and hanging-node interpolation C_e of
// one cell, written out node by node.  One cell per block, n^2 threads.
template <int K>
__global__ void __launch_bounds__((K + 1) * (K + 1))
    distribute_kernel(const int32_t* __restrict__ ent, const uint32_t* __restrict__ mask, int64_t nc,
                      OpTab<double, K + 1> tab, const double* __restrict__ x, double* __restrict__ out) {
  constexpr int N = K + 1, N2 = N * N, N3 = N2 * N;
  __shared__ double B[N3];
  const int64_t cell = blockIdx.x;
  const int ta = threadIdx.x % N, tb = threadIdx.x / N;
  const uint32_t m = mask[cell];
  double u[N];
#pragma unroll
  for (int c = 0; c < N; ++c) {
    const int s = node_slot(ta, tb, c, K);
    const int32_t e = ent[s * nc + cell];
    u[c] = e < 0 ? 0.0 : x[e + node_offset(ta, tb, c, K)];
  }
  const bool hang = mask_hanging(m);
  if (hang && hanging_line(m, 2, ta, tb, K)) interp<N, double, false>(tab.H, mask_sub(m, 2), u);
#pragma unroll
  for (int c = 0; c < N; ++c) B[c * N2 + tb * N + ta] = u[c];
  __syncthreads();
  // y-lines (x = ta, z = tb)
#pragma unroll
  for (int r = 0; r < N; ++r) u[r] = B[tb * N2 + r * N + ta];
  if (hang && hanging_line(m, 1, ta, tb, K)) interp<N, double, false>(tab.H, mask_sub(m, 1), u);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < N; ++r) B[tb * N2 + r * N + ta] = u[r];
  __syncthreads();
  // x-lines (y = ta, z = tb)
#pragma unroll
  for (int r = 0; r < N; ++r) u[r] = B[tb * N2 + ta * N + r];
  if (hang && hanging_line(m, 0, ta, tb, K)) interp<N, double, false>(tab.H, mask_sub(m, 0), u);
#pragma unroll
  for (int r = 0; r < N; ++r) out[cell * N3 + tb * N2 + ta * N + r] = u[r];
}

// Load vector b_e = int_e f phi (Gauss (k+1)^3), then C_e^T and scatter.
// One cell per block, n^2 threads; f = const or a sum of Gaussians.
template <int K>
__global__ void __launch_bounds__((K + 1) * (K + 1))
    rhs_kernel(const int32_t* __restrict__ ent, const uint32_t* __restrict__ mask,
               const int32_t* __restrict__ cell_ijk, int64_t nc, double h0, double lo, OpTab<double, K + 1> tab,
               Gauss1D<K + 1> g, int kind, const double* __restrict__ params, int n_terms, double* __restrict__ b,
               int nv, const double* __restrict__ geo, int n0, const int32_t* __restrict__ cells) {
  constexpr int N = K + 1, N2 = N * N, N3 = N2 * N;
  __shared__ double B0[N3];
  const int64_t cell = cells ? cells[blockIdx.x] : blockIdx.x;  // cells: one colour (deterministic mode)
  const int v = blockIdx.y;
  const int ta = threadIdx.x % N, tb = threadIdx.x / N;
  const uint32_t m = mask[cell];
  const int lev = mask_level(m);
  const double h = ldexp(h0, -lev);
  const double x0 = lo + h * cell_ijk[3 * cell + 0];
  const double y0 = lo + h * cell_ijk[3 * cell + 1];
  const double z0 = lo + h * cell_ijk[3 * cell + 2];
  // z-line of quadrature points (qx = ta, qy = tb): weighted f values
  double gz[N];
  CellGeo<double> cg{};
  if (geo) cg = cell_geo<double>(geo, cell_ijk, cell, lev, n0);
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double x = x0 + h * g.x[ta], y = y0 + h * g.x[tb], z = z0 + h * g.x[q];
    double vol = h * h * h;  // |det J| of the cell map
    if (geo) {  // mapped cell: physical point and |det J| from its map
      const double t1 = (cg.r[0] + g.x[ta]) * cg.scale, t2 = (cg.r[1] + g.x[tb]) * cg.scale,
                   t3 = (cg.r[2] + g.x[q]) * cg.scale;
      double X[3], J[3][3];
      geo_point<double>(cg.A, t1, t2, t3, X);
      geo_jacobian<double>(cg.A, t1, t2, t3, J);
      x = X[0];
      y = X[1];
      z = X[2];
      vol = (J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
             J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0])) *
            cg.scale * cg.scale * cg.scale;
      vol = vol < 0 ? -vol : vol;
    }
    double f = 0.0;
    if (kind == 0) {
      f = params[0];
    } else if (kind == 2) {
      f = params[0] * sin(params[1] * x) * sin(params[1] * y) * sin(params[1] * z);
    } else {
      const double* p = params + static_cast<int64_t>(v) * n_terms * 5;
      for (int t = 0; t < n_terms; ++t) {
        double dx = x - p[5 * t], dy = y - p[5 * t + 1], dz = z - p[5 * t + 2], w = p[5 * t + 3];
        f += p[5 * t + 4] * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * w * w));
      }
    }
    gz[q] = f * g.w[ta] * g.w[tb] * g.w[q] * vol;
  }
  // S^T along z: out[c] = sum_q S[q][c] gz[q]
  double u[N];
#pragma unroll
  for (int c = 0; c < N; ++c) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < N; ++q) s += g.S[q * N + c] * gz[q];
    u[c] = s;
  }
#pragma unroll
  for (int c = 0; c < N; ++c) B0[c * N2 + tb * N + ta] = u[c];  // (qx, qy, c)
  __syncthreads();
  // along y at (qx = ta, c = tb)
#pragma unroll
  for (int r = 0; r < N; ++r) gz[r] = B0[tb * N2 + r * N + ta];
#pragma unroll
  for (int bb = 0; bb < N; ++bb) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < N; ++q) s += g.S[q * N + bb] * gz[q];
    u[bb] = s;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < N; ++r) B0[tb * N2 + r * N + ta] = u[r];  // (qx, b, c)
  __syncthreads();
  // along x at (b = ta, c = tb)
#pragma unroll
  for (int r = 0; r < N; ++r) gz[r] = B0[tb * N2 + ta * N + r];
#pragma unroll
  for (int aa = 0; aa < N; ++aa) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < N; ++q) s += g.S[q * N + aa] * gz[q];
    u[aa] = s;
  }
  const bool hang = mask_hanging(m);
  if (hang && hanging_line(m, 0, ta, tb, K)) interp<N, double, true>(tab.H, mask_sub(m, 0), u);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < N; ++r) B0[tb * N2 + ta * N + r] = u[r];  // (a, b, c)
  __syncthreads();
  // z-lines (x = ta, y = tb): transposed z
#pragma unroll
  for (int r = 0; r < N; ++r) u[r] = B0[r * N2 + tb * N + ta];
  if (hang && hanging_line(m, 2, ta, tb, K)) interp<N, double, true>(tab.H, mask_sub(m, 2), u);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < N; ++r) B0[r * N2 + tb * N + ta] = u[r];
  __syncthreads();
  // y-lines (x = ta, z = tb): transposed y, scatter
#pragma unroll
  for (int r = 0; r < N; ++r) u[r] = B0[tb * N2 + r * N + ta];
  if (hang && hanging_line(m, 1, ta, tb, K)) interp<N, double, true>(tab.H, mask_sub(m, 1), u);
  scatter_yline<K>(ent, nc, cell, ta, tb, u, b, nv, v, cells != nullptr);
}

}  // namespace mfmg

namespace mfmg {

// ---------------------------------------------------------------------------
// Intergrid transfer (Section 3.5, Eq. eq:impl:loop:categorized): one coarse
// cell (transfer group) per block.  Prolongation:
//   coarse gather G_c with constraints C_c (in-place interpolation),
//   category prolongation P (three 1D sweeps; identity category: none),
//   weights W, scatter S_f.
// Restriction is the transpose of every step.  The weights: the paper's W
// divides each fine value by the number of groups that reach it, so that the
// groups' equal contributions sum to it once.  Here W is 1 on one owner
// (fine cell, slot) pair per fine entity and 0 elsewhere (and on constrained
// fine DoFs): the same operator, and the prolongation writes each fine DoF
// from one block with a plain read-modify-write instead of atomics.
//
// Lattice of a group: NF nodes per axis.  Refinement category: NF = 2k+1
// nodes covering the 8 children (child along an axis = node index >= k);
// polynomial category: NF = k_f+1; identity: NF = NC, no sweeps.
//
// Several interleaved vectors are handled VB at a time: the vector index is
// the fastest one of the threads and of the LDS arrays ([node][VB]), so the
// VB values of a DoF, adjacent in memory, are read and written by adjacent
// threads.  VB is the largest power of two <= 8 whose arrays fit 32 KB.
constexpr int TR_THREADS = 256;

template <int NF, int NC, typename T>
constexpr int transfer_vb() {
  constexpr int per = (NC * NC * NC + NF * NC * NC + NF * NF * NC + NF * NF * NF) * static_cast<int>(sizeof(T));
  return per * 8 <= 32768 ? 8 : per * 4 <= 32768 ? 4 : per * 2 <= 32768 ? 2 : 1;
}

// in-place hanging-node interpolation of the coarse cell's node values
// X[node][VB] (vectors vv < nb)
template <int KC, int VB, typename T>
__device__ __forceinline__ void constraints_lds(T* X, uint32_t m, const T (&H)[2][(KC + 1) * (KC + 1)],
                                                bool trans, int nb) {
  constexpr int N = KC + 1, N2 = N * N;
  for (int d = 0; d < 3; ++d) {
    __syncthreads();
    const int s = mask_sub(m, d);
    for (int t = threadIdx.x; t < N2 * nb; t += blockDim.x) {
      const int line = t / nb, vv = t - line * nb;
      const int p = line % N, q = line / N;
      if (!hanging_line(m, d, p, q, KC)) continue;
      T u[N];
      const int stride = d == 0 ? 1 : d == 1 ? N : N2;
      const int base = d == 0 ? p * N + q * N2 : d == 1 ? p + q * N2 : p + q * N;
#pragma unroll
      for (int r = 0; r < N; ++r) u[r] = X[(base + r * stride) * VB + vv];
      if (trans) interp<N, T, true>(H, s, u);
      else interp<N, T, false>(H, s, u);
#pragma unroll
      for (int r = 0; r < N; ++r) X[(base + r * stride) * VB + vv] = u[r];
    }
  }
  __syncthreads();
}

// out (NO along axis d) = P (NO x NI) applied along axis d of `in`; the
// other two axes (in increasing order) have extents na, nb in both; layout x
// fastest, then the VB vectors innermost
template <int NI, int NO, int VB, typename T, bool TRANS>
__device__ __forceinline__ void sweep_lds(const T* in, T* out, const T* __restrict__ P, int d, int na, int nb,
                                          int nvb) {
  const int lines = na * nb;
  for (int t = threadIdx.x; t < lines * nvb; t += blockDim.x) {
    const int line = t / nvb, vv = t - line * nvb;
    const int p = line % na, q = line / na;
    int sin, sout, bin, bout;
    if (d == 0) { sin = 1; sout = 1; bin = (p + q * na) * NI; bout = (p + q * na) * NO; }
    else if (d == 1) { sin = na; sout = na; bin = p + q * na * NI; bout = p + q * na * NO; }
    else { sin = na * nb; sout = na * nb; bin = p + q * na; bout = p + q * na; }
    T u[NI];
#pragma unroll
    for (int r = 0; r < NI; ++r) u[r] = in[(bin + r * sin) * VB + vv];
#pragma unroll
    for (int i = 0; i < NO; ++i) {
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < NI; ++j) acc += (TRANS ? P[j * NO + i] : P[i * NI + j]) * u[j];
      out[(bout + i * sout) * VB + vv] = acc;
    }
  }
}

// fine lattice node I (per axis) -> (child bit, local node)
template <int KF, int NF>
__device__ __forceinline__ void lattice_local(int I, int& child, int& a) {
  if constexpr (NF == 2 * KF + 1) {
    child = I >= KF ? 1 : 0;
    a = I - child * KF;
  } else {
    child = 0;
    a = I;
  }
}

template <int KF, int KC, int NF, typename S, typename T>
__global__ void __launch_bounds__(TR_THREADS)
    prolongate_kernel(const int32_t* __restrict__ fent, int64_t nfc, const int32_t* __restrict__ cent,
                      const uint32_t* __restrict__ cmask, int64_t ncc, const int32_t* __restrict__ group_coarse,
                      const int32_t* __restrict__ group_fine, int64_t gstride, int nchild,
                      const uint8_t* __restrict__ valence, TrTab<T, NF, KC + 1> tab, const S* __restrict__ src,
                      S* __restrict__ dst, int nv) {
  constexpr int NC = KC + 1, NC3 = NC * NC * NC, NF3 = NF * NF * NF;
  constexpr bool IDENT = (NF == NC) && (KF == KC);
  constexpr int VB = transfer_vb<NF, NC, T>();
  __shared__ T X[NC3 * VB];
  __shared__ T Y1[IDENT ? 1 : NF * NC * NC * VB];
  __shared__ T Y2[IDENT ? 1 : NF * NF * NC * VB];
  __shared__ T Y3[IDENT ? 1 : NF3 * VB];
  const int64_t g = blockIdx.x;
  const int64_t cc = group_coarse[g];
  const uint32_t mc = cmask[cc];
  for (int v0 = 0; v0 < nv; v0 += VB) {
    const int nb = nv - v0 < VB ? nv - v0 : VB;
    if (v0 > 0) __syncthreads();
    for (int t = threadIdx.x; t < NC3 * nb; t += blockDim.x) {
      const int i = t / nb, vv = t - i * nb;
      const int a = i % NC, b = (i / NC) % NC, c = i / (NC * NC);
      const int s = node_slot(a, b, c, KC);
      const int32_t e = cent[s * ncc + cc];
      X[i * VB + vv] =
          e < 0 ? T(0) : load_as<T>(src[static_cast<int64_t>(e + node_offset(a, b, c, KC)) * nv + v0 + vv]);
    }
    if (mask_hanging(mc)) constraints_lds<KC, VB, T>(X, mc, tab.H, false, nb);
    else __syncthreads();
    const T* Y = X;
    if constexpr (!IDENT) {
      sweep_lds<NC, NF, VB, T, false>(X, Y1, tab.P, 0, NC, NC, nb);
      __syncthreads();
      sweep_lds<NC, NF, VB, T, false>(Y1, Y2, tab.P, 1, NF, NC, nb);
      __syncthreads();
      sweep_lds<NC, NF, VB, T, false>(Y2, Y3, tab.P, 2, NF, NF, nb);
      __syncthreads();
      Y = Y3;
    }
    for (int t = threadIdx.x; t < NF3 * nb; t += blockDim.x) {
      const int i = t / nb, vv = t - i * nb;
      const int I = i % NF, J = (i / NF) % NF, L = i / (NF * NF);
      int cx, cy, cz, a, b, c;
      lattice_local<KF, NF>(I, cx, a);
      lattice_local<KF, NF>(J, cy, b);
      lattice_local<KF, NF>(L, cz, c);
      const int child = nchild == 8 ? cx + 2 * cy + 4 * cz : 0;
      const int64_t f = group_fine[child * gstride + g];
      const int s = node_slot(a, b, c, KF);
      // one (cell, slot) pair owns each fine entity: a plain read-modify-write
      if (!(valence[s * nfc + f] & TRANSFER_OWNER)) continue;
      const int32_t e = fent[s * nfc + f];
      const int64_t idx = static_cast<int64_t>(e + node_offset(a, b, c, KF)) * nv + v0 + vv;
      add_to<S, T>(&dst[idx], Y[i * VB + vv], true);
    }
  }
}

template <int KF, int KC, int NF, typename S, typename T>
__global__ void __launch_bounds__(TR_THREADS)
    restrict_kernel(const int32_t* __restrict__ fent, int64_t nfc, const int32_t* __restrict__ cent,
                    const uint32_t* __restrict__ cmask, int64_t ncc, const int32_t* __restrict__ group_coarse,
                    const int32_t* __restrict__ group_fine, int64_t gstride, int nchild,
                    const uint8_t* __restrict__ valence, TrTab<T, NF, KC + 1> tab, const S* __restrict__ src,
                    S* __restrict__ dst, int nv, bool plain) {
  constexpr int NC = KC + 1, NC3 = NC * NC * NC, NF3 = NF * NF * NF;
  constexpr bool IDENT = (NF == NC) && (KF == KC);
  constexpr int VB = transfer_vb<NF, NC, T>();
  __shared__ T X[NC3 * VB];
  __shared__ T Y1[IDENT ? 1 : NF * NC * NC * VB];
  __shared__ T Y2[IDENT ? 1 : NF * NF * NC * VB];
  __shared__ T Y3[IDENT ? 1 : NF3 * VB];
  const int64_t g = blockIdx.x;
  const int64_t cc = group_coarse[g];
  const uint32_t mc = cmask[cc];
  for (int v0 = 0; v0 < nv; v0 += VB) {
    const int nb = nv - v0 < VB ? nv - v0 : VB;
    if (v0 > 0) __syncthreads();
    T* Yw = IDENT ? X : Y3;
    for (int t = threadIdx.x; t < NF3 * nb; t += blockDim.x) {
      const int i = t / nb, vv = t - i * nb;
      const int I = i % NF, J = (i / NF) % NF, L = i / (NF * NF);
      int cx, cy, cz, a, b, c;
      lattice_local<KF, NF>(I, cx, a);
      lattice_local<KF, NF>(J, cy, b);
      lattice_local<KF, NF>(L, cz, c);
      const int child = nchild == 8 ? cx + 2 * cy + 4 * cz : 0;
      const int64_t f = group_fine[child * gstride + g];
      const int s = node_slot(a, b, c, KF);
      T y = T(0);
      if (valence[s * nfc + f] & TRANSFER_OWNER) {  // each fine value enters once
        const int32_t e = fent[s * nfc + f];
        y = load_as<T>(src[static_cast<int64_t>(e + node_offset(a, b, c, KF)) * nv + v0 + vv]);
      }
      Yw[i * VB + vv] = y;
    }
    __syncthreads();
    if constexpr (!IDENT) {
      sweep_lds<NF, NC, VB, T, true>(Y3, Y2, tab.P, 2, NF, NF, nb);
      __syncthreads();
      sweep_lds<NF, NC, VB, T, true>(Y2, Y1, tab.P, 1, NF, NC, nb);
      __syncthreads();
      sweep_lds<NF, NC, VB, T, true>(Y1, X, tab.P, 0, NC, NC, nb);
      __syncthreads();
    }
    if (mask_hanging(mc)) constraints_lds<KC, VB, T>(X, mc, tab.H, true, nb);
    for (int t = threadIdx.x; t < NC3 * nb; t += blockDim.x) {
      const int i = t / nb, vv = t - i * nb;
      const int a = i % NC, b = (i / NC) % NC, c = i / (NC * NC);
      const int s = node_slot(a, b, c, KC);
      const int32_t e = cent[s * ncc + cc];
      if (e < 0) continue;
      add_to<S, T>(&dst[static_cast<int64_t>(e + node_offset(a, b, c, KC)) * nv + v0 + vv], X[i * VB + vv],
                   plain || s == 26);
    }
  }
}

// ---------------------------------------------------------------------------
// vector kernels
constexpr int VEC_THREADS = 256;

inline unsigned grid_for(int64_t n, int per_thread = 1) {
  int64_t b = (n + static_cast<int64_t>(VEC_THREADS) * per_thread - 1) / (static_cast<int64_t>(VEC_THREADS) * per_thread);
  if (b < 1) b = 1;
  if (b > 1 << 20) b = 1 << 20;
  return static_cast<unsigned>(b);
}

__global__ void fill_zero_kernel(uint32_t* __restrict__ x, int64_t nwords) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < nwords;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    x[i] = 0u;
}

__global__ void fill_zero_bytes_kernel(uint8_t* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    x[i] = 0;
}

template <typename S>
__global__ void cheb_kernel(int64_t n_dofs, int nv, int first, typename Acc<S>::type c_dd,
                            typename Acc<S>::type c_r, const typename Acc<S>::type* __restrict__ t,
                            const S* __restrict__ b, const typename Acc<S>::type* __restrict__ dinv,
                            S* __restrict__ d, S* __restrict__ x) {
  using A = typename Acc<S>::type;
  const int64_t n = n_dofs * nv;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const A di = dinv[i / nv];
    A dn;
    if (first) {
      dn = c_r * di * load_as<A>(b[i]);
      x[i] = store_as<S>(dn);
    } else {
      dn = (c_dd != A(0) ? c_dd * load_as<A>(d[i]) : A(0)) + c_r * di * (load_as<A>(b[i]) - t[i]);
      x[i] = store_as<S>(load_as<A>(x[i]) + dn);
    }
    d[i] = store_as<S>(dn);
  }
}

template <typename S>
__global__ void residual_kernel(int64_t n, const S* __restrict__ b, const typename Acc<S>::type* __restrict__ t,
                                S* __restrict__ r) {
  using A = typename Acc<S>::type;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    r[i] = store_as<S>(load_as<A>(b[i]) - t[i]);
}

template <typename S>
__global__ void cast_from_f64_kernel(int64_t n, const double* __restrict__ src, S* __restrict__ dst) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[i] = store_as<S>(src[i]);
}

template <typename S>
__global__ void cast_to_f64_kernel(int64_t n, const S* __restrict__ src, double* __restrict__ dst) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[i] = load_as<double>(src[i]);
}

template <typename A, typename B>
__global__ void cast_kernel(int64_t n, const A* __restrict__ src, B* __restrict__ dst) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[i] = store_as<B>(load_as<float>(src[i]));
}

// copy between the active mesh and a local-smoothing level (Algorithm 1):
// dst[di[q]] = src[si[q]], n_vec interleaved values per DoF
template <typename A, typename B>
__global__ void copy_map_kernel(int64_t n, int nv, const int32_t* __restrict__ si, const int32_t* __restrict__ di,
                                const A* __restrict__ src, B* __restrict__ dst) {
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < n * nv;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t q = t / nv;
    const int64_t v = t - q * nv;
    dst[static_cast<int64_t>(di[q]) * nv + v] = store_as<B>(load_as<double>(src[static_cast<int64_t>(si[q]) * nv + v]));
  }
}

// refinement-edge DoFs of a local-smoothing level: zero inverse diagonal
__global__ void zero_entries_kernel(int64_t n, const int32_t* __restrict__ idx, double* __restrict__ a64,
                                    float* __restrict__ a32) {
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < n;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    a64[idx[t]] = 0.0;
    a32[idx[t]] = 0.0f;
  }
}

template <typename S>
__global__ void acc_to_storage_kernel(int64_t n, const typename Acc<S>::type* __restrict__ src,
                                      S* __restrict__ dst) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[i] = store_as<S>(src[i]);
}

template <typename A>
__global__ void inverse_diag_kernel(int64_t n, const double* __restrict__ diag, A* __restrict__ dinv) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dinv[i] = diag[i] != 0.0 ? static_cast<A>(1.0 / diag[i]) : A(0);
}

// one wavefront per row: acc[row] = sum_j Ainv[row, j] b[j]
template <typename S>
__global__ void __launch_bounds__(256)
    dense_matvec_kernel(int64_t n0, int nv, const typename Acc<S>::type* __restrict__ Ainv,
                        const S* __restrict__ b, S* __restrict__ x) {
  using A = typename Acc<S>::type;
  const int lane = threadIdx.x & 63;
  const int64_t row = static_cast<int64_t>(blockIdx.x) * (blockDim.x / 64) + threadIdx.x / 64;
  const int v = blockIdx.y;
  if (row >= n0) return;
  A s = A(0);
  for (int64_t j = lane; j < n0; j += 64) s += Ainv[row * n0 + j] * load_as<A>(b[j * nv + v]);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) x[row * nv + v] = store_as<S>(s);
}

// ---- FP64 reductions and CG updates ----------------------------------------
constexpr int DOT_BLOCKS = 512;

// per-vector partial dot products of interleaved vectors ([n][nv], nv <= 8):
// each thread accumulates all components of its DoFs, so that a block reads
// contiguous memory
__global__ void __launch_bounds__(256)
    dot_stage1(int64_t n_dofs, int nv, const double* __restrict__ a, const double* __restrict__ b,
               double* __restrict__ partial) {
  __shared__ double red[8][256];
  double s[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) s[v] = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n_dofs;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
#pragma unroll
    for (int v = 0; v < 8; ++v)
      if (v < nv) s[v] += a[i * nv + v] * b[i * nv + v];
  }
#pragma unroll
  for (int v = 0; v < 8; ++v) red[v][threadIdx.x] = s[v];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int v = 0; v < 8; ++v)
        if (v < nv) red[v][threadIdx.x] += red[v][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < nv) partial[threadIdx.x * DOT_BLOCKS + blockIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) dot_stage2(int nv, const double* __restrict__ partial,
                                                  double* __restrict__ result) {
  __shared__ double red[256];
  const int v = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < DOT_BLOCKS; i += blockDim.x) s += partial[v * DOT_BLOCKS + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) result[v] = red[0];
}

__global__ void cg_xr_kernel(int64_t n_dofs, int nv, const double* __restrict__ num, const double* __restrict__ den,
                             const double* __restrict__ p, const double* __restrict__ q, double* __restrict__ x,
                             double* __restrict__ r) {
  const int64_t n = n_dofs * nv;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int v = static_cast<int>(i % nv);
    const double alpha = den[v] != 0.0 ? num[v] / den[v] : 0.0;
    x[i] += alpha * p[i];
    r[i] -= alpha * q[i];
  }
}

__global__ void cg_p_kernel(int64_t n_dofs, int nv, const double* __restrict__ num, const double* __restrict__ sub,
                            const double* __restrict__ den, const double* __restrict__ z, double* __restrict__ p) {
  const int64_t n = n_dofs * nv;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int v = static_cast<int>(i % nv);
    const double beta = den[v] != 0.0 ? (num[v] - (sub ? sub[v] : 0.0)) / den[v] : 0.0;
    p[i] = z[i] + beta * p[i];
  }
}

// ===========================================================================
// host launchers
namespace {

void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(MFMG_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

void zero_bytes(void* p, int64_t bytes, hipStream_t s) {
  if (bytes <= 0) return;
  if (bytes % 4 == 0 && reinterpret_cast<uintptr_t>(p) % 4 == 0) {
    fill_zero_kernel<<<grid_for(bytes / 4, 4), VEC_THREADS, 0, s>>>(static_cast<uint32_t*>(p), bytes / 4);
  } else {
    fill_zero_bytes_kernel<<<grid_for(bytes, 4), VEC_THREADS, 0, s>>>(static_cast<uint8_t*>(p), bytes);
  }
  check_launch();
}

template <int K, typename S, int FK, int GEO, bool DET>
void vmult_run(const CellView& c, int nv, void* dst, const void* src, const FusedStep& f, hipStream_t s) {
  using T = typename Acc<S>::type;
  constexpr int N = K + 1;
  if (c.n_cells == 0) return;
  static const OpTab2<T, N> tab = make_optab2<T, N>();
  static const MapTab<T, N> mt = make_maptab<T, N>();
  if constexpr (GEO == 0) ensure_hg_table<T, N>();
  const T* geo = nullptr;
  if constexpr (GEO != 0) geo = static_cast<const T*>(sizeof(T) == 8 ? c.geo64 : c.geo32);
  // persistent blocks: as many as are resident on the device at once (a
  // multiple of 8, one share per XCD), at most one per batch
  static const int64_t resident = [] {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(&vmult_batch_kernel<K, S, T, FK, GEO, DET>), BATCH_WAVES * 64, 0) !=
            hipSuccess) {
      (void)hipGetLastError();
      return int64_t(0);
    }
    return static_cast<int64_t>(cus) * per_cu * BATCH_GRID_FACTOR;
  }();
  const int64_t nb = c.n_batches;
  int64_t blocks = 8 * ((nb * nv + 7) / 8);  // (several vectors: one block per (batch, vector) at most)
  if (resident >= 8 && blocks > resident / 8 * 8) blocks = resident / 8 * 8;
  if (blocks < 8 * nv) blocks = 8 * nv;  // every XCD runs all vectors of a batch together
  constexpr bool atom = (FK & FUSE_ATOMIC) != 0;
  constexpr bool into_dst = base_kind(FK) == FUSE_NONE;
  if (atom && c.n_shared > 0) {  // (the shared DoFs are the first n_shared)
    clear_shared_kernel<T><<<grid_for(c.n_shared), VEC_THREADS, 0, s>>>(
        c.n_shared, static_cast<T*>(into_dst ? dst : c.partial));
    check_launch();
  }
  vmult_batch_kernel<K, S, T, FK, GEO, DET><<<static_cast<unsigned>(blocks), BATCH_WAVES * 64, 0, s>>>(
      c.meta, c.batch_cell, c.batch_sh, c.batch_ex, c.sh_idx, nb, c.n_shared, c.h0, tab,
      static_cast<const S*>(src), static_cast<T*>(c.partial), static_cast<T*>(dst), nv, f, geo, c.ijk, c.geo_n0,
      mt);
  check_launch();
  if constexpr (atom && !into_dst) {
    if (c.n_shared > 0) {
      finish_shared_kernel<S, T, base_kind(FK)><<<grid_for(c.n_shared), VEC_THREADS, 0, s>>>(
          c.n_shared, static_cast<const T*>(c.partial), static_cast<T*>(dst), f);
      check_launch();
    }
  }
  if constexpr (!atom) {
    if (c.n_shared > 0) {
      const T* part = static_cast<const T*>(c.partial);  // (256-byte aligned: vector loads of NV values)
      T* out = static_cast<T*>(dst);
      const unsigned g = grid_for(c.n_shared);
      if (nv == 8) {
        reduce_shared_vec_kernel<S, T, FK, 8><<<g, VEC_THREADS, 0, s>>>(c.n_shared, c.red_off, c.red_idx, part, out, f);
      } else if (nv == 4) {
        reduce_shared_vec_kernel<S, T, FK, 4><<<g, VEC_THREADS, 0, s>>>(c.n_shared, c.red_off, c.red_idx, part, out, f);
      } else if (nv == 2) {
        reduce_shared_vec_kernel<S, T, FK, 2><<<g, VEC_THREADS, 0, s>>>(c.n_shared, c.red_off, c.red_idx, part, out, f);
      } else {
        reduce_shared_kernel<S, T, FK><<<grid_for(c.n_shared * nv), VEC_THREADS, 0, s>>>(
            c.n_shared, nv, c.red_off, c.red_idx, part, out, f);
      }
      check_launch();
    }
  }
}

// One vector: the shared DoFs' sums go out with global atomics, which run
// alongside the evaluation and replace the partial sums' write and the
// reduction's gathers.  Interleaved vectors keep the partial sums (their
// atomics would meet in one line, which measured slower), and so does the
// deterministic mode (their fixed order).
template <int K, typename S, int FK, int GEO, bool DET>
void vmult_kgd(const CellView& c, int nv, void* dst, const void* src, const FusedStep& f, hipStream_t s) {
  if constexpr (!DET) {
    if (nv == 1) {
      vmult_run<K, S, FK | FUSE_ATOMIC, GEO, false>(c, nv, dst, src, f, s);
      return;
    }
  }
  vmult_run<K, S, FK, GEO, DET>(c, nv, dst, src, f, s);
}

template <int K, typename S, int FK, int GEO>
void vmult_kg(const CellView& c, int nv, void* dst, const void* src, const FusedStep& f, hipStream_t s) {
  if (c.deterministic) vmult_kgd<K, S, FK, GEO, true>(c, nv, dst, src, f, s);
  else vmult_kgd<K, S, FK, GEO, false>(c, nv, dst, src, f, s);
}

template <int K, typename S, int FK>
void vmult_k(const CellView& c, int nv, void* dst, const void* src, const FusedStep& f, hipStream_t s) {
  if (c.geo64) vmult_kg<K, S, FK, 1>(c, nv, dst, src, f, s);
  else vmult_kg<K, S, FK, 0>(c, nv, dst, src, f, s);
}

template <int K, typename S>
void vmult_kf(const CellView& c, int nv, void* dst, const void* src, const FusedStep& f, hipStream_t s) {
  switch (f.kind) {
    case FUSE_NONE: vmult_k<K, S, FUSE_NONE>(c, nv, dst, src, f, s); break;
    case FUSE_CHEB: vmult_k<K, S, FUSE_CHEB>(c, nv, dst, src, f, s); break;
    case FUSE_RESIDUAL: vmult_k<K, S, FUSE_RESIDUAL>(c, nv, dst, src, f, s); break;
    default: throw Error(MFMG_ERR_INVALID_ARG, "fused step");
  }
}

template <typename S>
void vmult_s(const CellView& c, int nv, void* dst, const void* src, const FusedStep& f, hipStream_t s) {
  switch (c.k) {
    case 1: vmult_kf<1, S>(c, nv, dst, src, f, s); break;
    case 2: vmult_kf<2, S>(c, nv, dst, src, f, s); break;
    case 3: vmult_kf<3, S>(c, nv, dst, src, f, s); break;
    case 4: vmult_kf<4, S>(c, nv, dst, src, f, s); break;
    case 5: vmult_kf<5, S>(c, nv, dst, src, f, s); break;
    case 6: vmult_kf<6, S>(c, nv, dst, src, f, s); break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "degree");
  }
}

// One launch over all cells (cells = NULL: block i is cell i), or in the
// deterministic mode one launch per colour over that colour's cell list.
template <typename F>
void for_colours(const CellView& c, F launch) {
  if (!c.deterministic) {
    launch(static_cast<unsigned>(c.n_cells), static_cast<const int32_t*>(nullptr));
    return;
  }
  for (int k = 0; k < c.n_colors; ++k) {
    const int64_t n = c.color_off[k + 1] - c.color_off[k];
    if (n > 0) launch(static_cast<unsigned>(n), c.color_cells + c.color_off[k]);
  }
}

template <int K>
void diag_k(const CellView& c, double* diag, hipStream_t s) {
  constexpr int N = K + 1;
  zero_bytes(diag, c.n_dofs * 8, s);
  if (c.n_cells == 0) return;
  if (c.geo64) {
    static const MapTab<double, N> mt = make_maptab<double, N>();
    static const OpTab2<double, N> tab2 = make_optab2<double, N>();
    static const DiagTab<double, N> dt = [] {
      const Tables1D& t = tables(N - 1);
      DiagTab<double, N> r;
      for (int q = 0; q < N; ++q)
        for (int a = 0; a < N; ++a) {
          const double sv = t.S[q * N + a], dv = lagrange_deriv(t.nodes, a, t.qp[q]);
          r.E[q * N + a] = sv * sv;
          r.F[q * N + a] = dv * dv;
          r.X[q * N + a] = dv * sv;
        }
      return r;
    }();
    const double* geo = static_cast<const double*>(c.geo64);
    for_colours(c, [&](unsigned n, const int32_t* cells) {
      diag_mapped_direct_kernel<K><<<n, N * N, 0, s>>>(c.ent, c.mask, c.n_cells, geo, c.ijk, c.geo_n0, mt, dt, diag,
                                                       cells);
      check_launch();
      diag_mapped_kernel<K><<<n, N * N, 0, s>>>(c.ent, c.mask, c.n_cells, geo, c.ijk, c.geo_n0, mt, tab2, diag,
                                                cells);
      check_launch();
    });
    return;
  }
  static const OpTab<double, N> tab = make_optab<double, N>();
  for_colours(c, [&](unsigned n, const int32_t* cells) {
    diag_kernel<K><<<n, N * N, 0, s>>>(c.ent, c.mask, c.n_cells, c.h0, tab, diag, cells);
    check_launch();
  });
}

template <int K>
void rhs_k(const CellView& c, int kind, const double* params, int n_terms, int nv, double* b, hipStream_t s) {
  constexpr int N = K + 1;
  zero_bytes(b, c.n_dofs * nv * 8, s);
  if (c.n_cells == 0) return;
  static const OpTab<double, N> tab = make_optab<double, N>();
  static const Gauss1D<N> g = make_gauss<N>();
  for_colours(c, [&](unsigned n, const int32_t* cells) {
    dim3 grid(n, nv);
    rhs_kernel<K><<<grid, N * N, 0, s>>>(c.ent, c.mask, c.ijk, c.n_cells, c.h0, c.lo, tab, g, kind, params,
                                         n_terms, b, nv, static_cast<const double*>(c.geo64), c.geo_n0, cells);
    check_launch();
  });
}

template <typename T, int NF, int NC>
TrTab<T, NF, NC> make_trtab(int kf, int kc) {
  TrTab<T, NF, NC> t;
  const Tables1D& tc = tables(kc);
  for (int i = 0; i < NC * NC; ++i) {
    t.H[0][i] = static_cast<T>(tc.H[0][i]);
    t.H[1][i] = static_cast<T>(tc.H[1][i]);
  }
  if (kf == kc && NF == 2 * kc + 1) {
    for (int i = 0; i < NF * NC; ++i) t.P[i] = static_cast<T>(tc.T[i]);
  } else if (kf != kc && NF == 2 * kf + 1) {
    std::vector<double> P = hp_transfer_matrix(kf, kc);
    for (int i = 0; i < NF * NC; ++i) t.P[i] = static_cast<T>(P[i]);
  } else if (kf != kc) {
    std::vector<double> P = p_transfer_matrix(kf, kc);
    for (int i = 0; i < NF * NC; ++i) t.P[i] = static_cast<T>(P[i]);
  } else {
    for (int i = 0; i < NF * NC; ++i) t.P[i] = static_cast<T>((i / NC) == (i % NC) ? 1.0 : 0.0);
  }
  return t;
}

template <int KF, int KC, int NF, typename S>
void transfer_launch(bool prolong, const CellView& f, const CellView& c, const TransferView& t,
                     const int32_t* gc, const int32_t* gf, int64_t ng, int nchild, int nv, void* dst,
                     const void* src, hipStream_t s) {
  using T = typename Acc<S>::type;
  if (ng == 0) return;
  static const TrTab<T, NF, KC + 1> tab = make_trtab<T, NF, KC + 1>(KF, KC);
  if (prolong) {  // each fine DoF has one writer: no colouring needed
    prolongate_kernel<KF, KC, NF, S, T><<<static_cast<unsigned>(ng), TR_THREADS, 0, s>>>(
        f.ent, f.n_cells, c.ent, c.mask, c.n_cells, gc, gf, ng, nchild, t.valence, tab,
        static_cast<const S*>(src), static_cast<S*>(dst), nv);
    check_launch();
    return;
  }
  // restriction: one launch, or in the deterministic mode one per colour of
  // the group list (plain adds into the coarse DoFs)
  const int64_t* off = nchild == 1 ? t.ident_off : t.refined_off;
  const int n_col = nchild == 1 ? t.n_ident_colors : t.n_refined_colors;
  const int64_t whole[2] = {0, ng};
  const bool det = t.deterministic && off != nullptr;
  const int64_t* o = det ? off : whole;
  for (int k = 0; k < (det ? n_col : 1); ++k) {
    const int64_t n = o[k + 1] - o[k];
    if (n == 0) continue;
    restrict_kernel<KF, KC, NF, S, T><<<static_cast<unsigned>(n), TR_THREADS, 0, s>>>(
        f.ent, f.n_cells, c.ent, c.mask, c.n_cells, gc + o[k], gf + o[k], ng, nchild, t.valence, tab,
        static_cast<const S*>(src), static_cast<S*>(dst), nv, det);
    check_launch();
  }
}

template <int K, typename S>
void transfer_h(bool prolong, const CellView& f, const CellView& c, const TransferView& t, int nv, void* dst,
                const void* src, hipStream_t s) {
  transfer_launch<K, K, K + 1, S>(prolong, f, c, t, t.ident_coarse, t.ident_fine, t.n_ident, 1, nv, dst, src, s);
  transfer_launch<K, K, 2 * K + 1, S>(prolong, f, c, t, t.refined_coarse, t.refined_fine, t.n_refined, 8, nv,
                                     dst, src, s);
}

// geometric and polynomial coarsening in one step: identity pairs change the
// degree only, refined groups change both
template <int KF, int KC, typename S>
void transfer_hp(bool prolong, const CellView& f, const CellView& c, const TransferView& t, int nv, void* dst,
                 const void* src, hipStream_t s) {
  transfer_launch<KF, KC, KF + 1, S>(prolong, f, c, t, t.ident_coarse, t.ident_fine, t.n_ident, 1, nv, dst, src, s);
  transfer_launch<KF, KC, 2 * KF + 1, S>(prolong, f, c, t, t.refined_coarse, t.refined_fine, t.n_refined, 8, nv,
                                         dst, src, s);
}

template <typename S>
void transfer_s(bool prolong, const CellView& f, const CellView& c, const TransferView& t, int nv, void* dst,
                const void* src, hipStream_t s) {
  if (!t.polynomial && f.k != c.k) {
    switch (f.k * 10 + c.k) {
      case 21: transfer_hp<2, 1, S>(prolong, f, c, t, nv, dst, src, s); break;
      case 31: transfer_hp<3, 1, S>(prolong, f, c, t, nv, dst, src, s); break;
      case 42: transfer_hp<4, 2, S>(prolong, f, c, t, nv, dst, src, s); break;
      case 52: transfer_hp<5, 2, S>(prolong, f, c, t, nv, dst, src, s); break;
      case 63: transfer_hp<6, 3, S>(prolong, f, c, t, nv, dst, src, s); break;
      default: throw Error(MFMG_ERR_UNSUPPORTED, "combined h and p transfer pair");
    }
    return;
  }
  if (!t.polynomial) {
    switch (f.k) {
      case 1: transfer_h<1, S>(prolong, f, c, t, nv, dst, src, s); break;
      case 2: transfer_h<2, S>(prolong, f, c, t, nv, dst, src, s); break;
      case 3: transfer_h<3, S>(prolong, f, c, t, nv, dst, src, s); break;
      case 4: transfer_h<4, S>(prolong, f, c, t, nv, dst, src, s); break;
      case 5: transfer_h<5, S>(prolong, f, c, t, nv, dst, src, s); break;
      case 6: transfer_h<6, S>(prolong, f, c, t, nv, dst, src, s); break;
      default: throw Error(MFMG_ERR_UNSUPPORTED, "degree");
    }
    return;
  }
  const int key = f.k * 10 + c.k;
  switch (key) {
#define MFMG_P(KF, KC)                                                                                  \
  case KF * 10 + KC:                                                                                   \
    transfer_launch<KF, KC, KF + 1, S>(prolong, f, c, t, t.ident_coarse, t.ident_fine, t.n_ident, 1, nv, dst, \
                                       src, s);                                                        \
    break;
    MFMG_P(2, 1)
    MFMG_P(3, 1)
    MFMG_P(4, 2)
    MFMG_P(5, 2)
    MFMG_P(6, 3)
#undef MFMG_P
    default:
      throw Error(MFMG_ERR_UNSUPPORTED, "polynomial transfer pair");
  }
}

}  // namespace

void launch_vmult_fused(const CellView& c, int dtype, int nv, void* dst, const void* src, const FusedStep& f,
                        hipStream_t s) {
  switch (dtype) {
    case MFMG_F64: vmult_s<double>(c, nv, dst, src, f, s); break;
    case MFMG_F32: vmult_s<float>(c, nv, dst, src, f, s); break;
    case MFMG_BF16: vmult_s<bf16>(c, nv, dst, src, f, s); break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "dtype");
  }
}

void launch_vmult(const CellView& c, int dtype, int nv, void* dst, const void* src, hipStream_t s) {
  launch_vmult_fused(c, dtype, nv, dst, src, FusedStep{}, s);
}

void launch_diagonal(const CellView& c, double* diag, hipStream_t s) {
  switch (c.k) {
    case 1: diag_k<1>(c, diag, s); break;
    case 2: diag_k<2>(c, diag, s); break;
    case 3: diag_k<3>(c, diag, s); break;
    case 4: diag_k<4>(c, diag, s); break;
    case 5: diag_k<5>(c, diag, s); break;
    case 6: diag_k<6>(c, diag, s); break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "degree");
  }
}

template <int K>
void distribute_k(const CellView& c, const double* x, double* out, hipStream_t s) {
  constexpr int N = K + 1;
  if (c.n_cells == 0) return;
  static const OpTab<double, N> tab = make_optab<double, N>();
  distribute_kernel<K><<<static_cast<unsigned>(c.n_cells), N * N, 0, s>>>(c.ent, c.mask, c.n_cells, tab, x, out);
  check_launch();
}

void launch_distribute(const CellView& c, const double* x, double* out, hipStream_t s) {
  switch (c.k) {
    case 1: distribute_k<1>(c, x, out, s); break;
    case 2: distribute_k<2>(c, x, out, s); break;
    case 3: distribute_k<3>(c, x, out, s); break;
    case 4: distribute_k<4>(c, x, out, s); break;
    case 5: distribute_k<5>(c, x, out, s); break;
    case 6: distribute_k<6>(c, x, out, s); break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "degree");
  }
}

void launch_rhs(const CellView& c, int kind, const double* params, int n_terms, int nv, double* b,
                hipStream_t s) {
  switch (c.k) {
    case 1: rhs_k<1>(c, kind, params, n_terms, nv, b, s); break;
    case 2: rhs_k<2>(c, kind, params, n_terms, nv, b, s); break;
    case 3: rhs_k<3>(c, kind, params, n_terms, nv, b, s); break;
    case 4: rhs_k<4>(c, kind, params, n_terms, nv, b, s); break;
    case 5: rhs_k<5>(c, kind, params, n_terms, nv, b, s); break;
    case 6: rhs_k<6>(c, kind, params, n_terms, nv, b, s); break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "degree");
  }
}

void launch_prolongate(const CellView& f, const CellView& c, const TransferView& t, int dtype, int nv, void* dst,
                       const void* src, hipStream_t s) {
  switch (dtype) {
    case MFMG_F64: transfer_s<double>(true, f, c, t, nv, dst, src, s); break;
    case MFMG_F32: transfer_s<float>(true, f, c, t, nv, dst, src, s); break;
    case MFMG_BF16: transfer_s<bf16>(true, f, c, t, nv, dst, src, s); break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "dtype");
  }
}

void launch_restrict(const CellView& f, const CellView& c, const TransferView& t, int dtype, int nv, void* dst,
                     const void* src, hipStream_t s) {
  switch (dtype) {
    case MFMG_F64: transfer_s<double>(false, f, c, t, nv, dst, src, s); break;
    case MFMG_F32: transfer_s<float>(false, f, c, t, nv, dst, src, s); break;
    case MFMG_BF16: transfer_s<bf16>(false, f, c, t, nv, dst, src, s); break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "dtype");
  }
}

void launch_fill(int, void* x, int64_t n_bytes, hipStream_t s) { zero_bytes(x, n_bytes, s); }

void launch_cheb_step(int dtype, int64_t n_dofs, int nv, bool first, double c_dd, double c_r, const void* t,
                      const void* b, const void* dinv, void* d, void* x, hipStream_t s) {
  const unsigned g = grid_for(n_dofs * nv);
  switch (dtype) {
    case MFMG_F64:
      cheb_kernel<double><<<g, VEC_THREADS, 0, s>>>(n_dofs, nv, first, c_dd, c_r, static_cast<const double*>(t),
                                                    static_cast<const double*>(b), static_cast<const double*>(dinv),
                                                    static_cast<double*>(d), static_cast<double*>(x));
      break;
    case MFMG_F32:
      cheb_kernel<float><<<g, VEC_THREADS, 0, s>>>(n_dofs, nv, first, static_cast<float>(c_dd),
                                                   static_cast<float>(c_r), static_cast<const float*>(t),
                                                   static_cast<const float*>(b), static_cast<const float*>(dinv),
                                                   static_cast<float*>(d), static_cast<float*>(x));
      break;
    case MFMG_BF16:
      cheb_kernel<bf16><<<g, VEC_THREADS, 0, s>>>(n_dofs, nv, first, static_cast<float>(c_dd),
                                                  static_cast<float>(c_r), static_cast<const float*>(t),
                                                  static_cast<const bf16*>(b), static_cast<const float*>(dinv),
                                                  static_cast<bf16*>(d), static_cast<bf16*>(x));
      break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "dtype");
  }
  check_launch();
}

void launch_residual_update(int dtype, int64_t n, const void* b, const void* t, void* r, hipStream_t s) {
  const unsigned g = grid_for(n);
  switch (dtype) {
    case MFMG_F64:
      residual_kernel<double><<<g, VEC_THREADS, 0, s>>>(n, static_cast<const double*>(b),
                                                        static_cast<const double*>(t), static_cast<double*>(r));
      break;
    case MFMG_F32:
      residual_kernel<float><<<g, VEC_THREADS, 0, s>>>(n, static_cast<const float*>(b),
                                                       static_cast<const float*>(t), static_cast<float*>(r));
      break;
    case MFMG_BF16:
      residual_kernel<bf16><<<g, VEC_THREADS, 0, s>>>(n, static_cast<const bf16*>(b), static_cast<const float*>(t),
                                                      static_cast<bf16*>(r));
      break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "dtype");
  }
  check_launch();
}

void launch_cast_from_f64(int dtype, int64_t n, const double* src, void* dst, hipStream_t s) {
  const unsigned g = grid_for(n);
  switch (dtype) {
    case MFMG_F64: cast_from_f64_kernel<double><<<g, VEC_THREADS, 0, s>>>(n, src, static_cast<double*>(dst)); break;
    case MFMG_F32: cast_from_f64_kernel<float><<<g, VEC_THREADS, 0, s>>>(n, src, static_cast<float*>(dst)); break;
    case MFMG_BF16: cast_from_f64_kernel<bf16><<<g, VEC_THREADS, 0, s>>>(n, src, static_cast<bf16*>(dst)); break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "dtype");
  }
  check_launch();
}

void launch_cast_to_f64(int dtype, int64_t n, const void* src, double* dst, hipStream_t s) {
  const unsigned g = grid_for(n);
  switch (dtype) {
    case MFMG_F64: cast_to_f64_kernel<double><<<g, VEC_THREADS, 0, s>>>(n, static_cast<const double*>(src), dst); break;
    case MFMG_F32: cast_to_f64_kernel<float><<<g, VEC_THREADS, 0, s>>>(n, static_cast<const float*>(src), dst); break;
    case MFMG_BF16: cast_to_f64_kernel<bf16><<<g, VEC_THREADS, 0, s>>>(n, static_cast<const bf16*>(src), dst); break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "dtype");
  }
  check_launch();
}

void launch_cast(int dtype_src, int dtype_dst, int64_t n, const void* src, void* dst, hipStream_t s) {
  if (dtype_src == MFMG_F64) { launch_cast_from_f64(dtype_dst, n, static_cast<const double*>(src), dst, s); return; }
  if (dtype_dst == MFMG_F64) { launch_cast_to_f64(dtype_src, n, src, static_cast<double*>(dst), s); return; }
  const unsigned g = grid_for(n);
  if (dtype_src == MFMG_F32 && dtype_dst == MFMG_BF16)
    cast_kernel<float, bf16><<<g, VEC_THREADS, 0, s>>>(n, static_cast<const float*>(src), static_cast<bf16*>(dst));
  else if (dtype_src == MFMG_BF16 && dtype_dst == MFMG_F32)
    cast_kernel<bf16, float><<<g, VEC_THREADS, 0, s>>>(n, static_cast<const bf16*>(src), static_cast<float*>(dst));
  else if (dtype_src == dtype_dst)
    (void)hipMemcpyAsync(dst, src, n * dtype_size(dtype_src), hipMemcpyDeviceToDevice, s);
  else
    throw Error(MFMG_ERR_UNSUPPORTED, "cast");
  check_launch();
}

namespace {
template <typename A>
void copy_map_to(int dtype_dst, int64_t n, int nv, const int32_t* si, const int32_t* di, const A* src, void* dst,
                 hipStream_t s) {
  const unsigned g = grid_for(n * nv);
  switch (dtype_dst) {
    case MFMG_F64: copy_map_kernel<A, double><<<g, VEC_THREADS, 0, s>>>(n, nv, si, di, src, static_cast<double*>(dst)); break;
    case MFMG_F32: copy_map_kernel<A, float><<<g, VEC_THREADS, 0, s>>>(n, nv, si, di, src, static_cast<float*>(dst)); break;
    case MFMG_BF16: copy_map_kernel<A, bf16><<<g, VEC_THREADS, 0, s>>>(n, nv, si, di, src, static_cast<bf16*>(dst)); break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "dtype");
  }
}
}  // namespace

void launch_copy_map(int dtype_src, int dtype_dst, int64_t n, int nv, const int32_t* src_idx, const int32_t* dst_idx,
                     const void* src, void* dst, hipStream_t s) {
  if (n == 0) return;
  switch (dtype_src) {
    case MFMG_F64: copy_map_to(dtype_dst, n, nv, src_idx, dst_idx, static_cast<const double*>(src), dst, s); break;
    case MFMG_F32: copy_map_to(dtype_dst, n, nv, src_idx, dst_idx, static_cast<const float*>(src), dst, s); break;
    case MFMG_BF16: copy_map_to(dtype_dst, n, nv, src_idx, dst_idx, static_cast<const bf16*>(src), dst, s); break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "dtype");
  }
  check_launch();
}

void launch_zero_entries(int64_t n, const int32_t* idx, double* a64, float* a32, hipStream_t s) {
  if (n == 0) return;
  zero_entries_kernel<<<grid_for(n), VEC_THREADS, 0, s>>>(n, idx, a64, a32);
  check_launch();
}

void launch_acc_to_storage(int dtype, int64_t n, const void* acc, void* dst, hipStream_t s) {
  const unsigned g = grid_for(n);
  switch (dtype) {
    case MFMG_F64:
      acc_to_storage_kernel<double><<<g, VEC_THREADS, 0, s>>>(n, static_cast<const double*>(acc),
                                                              static_cast<double*>(dst));
      break;
    case MFMG_F32:
      acc_to_storage_kernel<float><<<g, VEC_THREADS, 0, s>>>(n, static_cast<const float*>(acc),
                                                             static_cast<float*>(dst));
      break;
    case MFMG_BF16:
      acc_to_storage_kernel<bf16><<<g, VEC_THREADS, 0, s>>>(n, static_cast<const float*>(acc),
                                                            static_cast<bf16*>(dst));
      break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "dtype");
  }
  check_launch();
}

namespace {
__global__ void coef_check_kernel(int64_t n, const double* __restrict__ c, int* __restrict__ flag) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    if (!(c[i] >= 1e-30 && c[i] <= 1e30)) flag[0] = 1;
}

__global__ void coef_restrict_kernel(int64_t n_ident, const int32_t* __restrict__ ident_c,
                                     const int32_t* __restrict__ ident_f, int64_t n_ref,
                                     const int32_t* __restrict__ ref_c, const int32_t* __restrict__ ref_f,
                                     const double* __restrict__ cf, double* __restrict__ cc) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n_ident + n_ref;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (i < n_ident) {
      cc[ident_c[i]] = cf[ident_f[i]];
    } else {
      const int64_t r = i - n_ident;
      double sum = 0.0;
      for (int ch = 0; ch < 8; ++ch) sum += cf[ref_f[ch * n_ref + r]];
      cc[ref_c[r]] = sum / 8.0;
    }
  }
}

__global__ void coef_apply_kernel(int64_t n, const double* __restrict__ c, uint32_t* __restrict__ mask,
                                  CellMeta* __restrict__ meta) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint32_t m = (mask[i] & ~MASK_COEF_BITS) | coef_bits(c[i]);
    mask[i] = m;
    meta[i].mask = m;
  }
}
}  // namespace

void launch_coef_check(int64_t n, const double* c, int* flag, hipStream_t s) {
  if (n == 0) return;
  coef_check_kernel<<<grid_for(n), VEC_THREADS, 0, s>>>(n, c, flag);
  check_launch();
}

void launch_coef_restrict(const TransferView& t, const double* c_fine, double* c_coarse, hipStream_t s) {
  const int64_t n = t.n_ident + t.n_refined;
  if (n == 0) return;
  coef_restrict_kernel<<<grid_for(n), VEC_THREADS, 0, s>>>(t.n_ident, t.ident_coarse, t.ident_fine, t.n_refined,
                                                         t.refined_coarse, t.refined_fine, c_fine, c_coarse);
  check_launch();
}

void launch_coef_apply(int64_t n_cells, const double* c, uint32_t* mask, CellMeta* meta, hipStream_t s) {
  if (n_cells == 0) return;
  coef_apply_kernel<<<grid_for(n_cells), VEC_THREADS, 0, s>>>(n_cells, c, mask, meta);
  check_launch();
}

void launch_inverse_diag(int dtype, int64_t n, const double* diag, void* dinv, hipStream_t s) {
  const unsigned g = grid_for(n);
  if (dtype == MFMG_F64)
    inverse_diag_kernel<double><<<g, VEC_THREADS, 0, s>>>(n, diag, static_cast<double*>(dinv));
  else
    inverse_diag_kernel<float><<<g, VEC_THREADS, 0, s>>>(n, diag, static_cast<float*>(dinv));
  check_launch();
}

void launch_dense_matvec(int dtype, int64_t n0, int nv, const void* Ainv, const void* b, void* x, void*,
                         hipStream_t s) {
  if (n0 == 0) return;
  dim3 grid(static_cast<unsigned>((n0 + 3) / 4), nv);
  switch (dtype) {
    case MFMG_F64:
      dense_matvec_kernel<double><<<grid, 256, 0, s>>>(n0, nv, static_cast<const double*>(Ainv),
                                                       static_cast<const double*>(b), static_cast<double*>(x));
      break;
    case MFMG_F32:
      dense_matvec_kernel<float><<<grid, 256, 0, s>>>(n0, nv, static_cast<const float*>(Ainv),
                                                      static_cast<const float*>(b), static_cast<float*>(x));
      break;
    case MFMG_BF16:
      dense_matvec_kernel<bf16><<<grid, 256, 0, s>>>(n0, nv, static_cast<const float*>(Ainv),
                                                     static_cast<const bf16*>(b), static_cast<bf16*>(x));
      break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "dtype");
  }
  check_launch();
}

int dot_partials_needed() { return DOT_BLOCKS; }

void launch_dot(int64_t n_dofs, int nv, const double* a, const double* b, double* partial, double* result,
                hipStream_t s) {
  if (nv < 1 || nv > 8) throw Error(MFMG_ERR_INVALID_ARG, "dot: n_vec must be in [1, 8]");
  dot_stage1<<<DOT_BLOCKS, 256, 0, s>>>(n_dofs, nv, a, b, partial);
  check_launch();
  dot_stage2<<<nv, 256, 0, s>>>(nv, partial, result);
  check_launch();
}

void launch_cg_update_xr(int64_t n_dofs, int nv, const double* num, const double* den, const double* p,
                         const double* q, double* x, double* r, hipStream_t s) {
  cg_xr_kernel<<<grid_for(n_dofs * nv), VEC_THREADS, 0, s>>>(n_dofs, nv, num, den, p, q, x, r);
  check_launch();
}

void launch_cg_update_p(int64_t n_dofs, int nv, const double* num, const double* sub, const double* den,
                        const double* z, double* p, hipStream_t s) {
  cg_p_kernel<<<grid_for(n_dofs * nv), VEC_THREADS, 0, s>>>(n_dofs, nv, num, sub, den, z, p);
  check_launch();
}

}  // namespace mfmg
