// Learned coarse-grid correction: a per-coarse-cell MLP replacing the exact
// coarse solve of Algorithm 2 (level 0), trained on coarse right-hand sides
// recorded from the solver itself.  FP32 arithmetic.
//
// Network: in = nq + 3 (coarse RHS at the cell's nq = (k+1)^3 nodes divided
// by s = ||b0||_2, cell centre), two hidden layers of width 64 with
// GELU(z) = z Phi(z), linear output of nq (correction / s).  Node values of
// several cells are averaged; Dirichlet nodes are 0.  Flat parameters:
// W1 (in x 64), b1, W2 (64 x 64), b2, W3 (64 x nq), b3.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <random>

#include "net.hpp"
#include "slots.hpp"

namespace mfmg {

namespace {

constexpr int HID = 64;
constexpr int ROWS_PER_BLOCK = 64;

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_df(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(MFMG_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

// Y[r][j] = sum_k X[r][k] W[k][j] + b[j]; Z = Y (pre-activation), H = act(Y)
__global__ void __launch_bounds__(256)
    linear_fwd(int rows, int K, int N, const float* __restrict__ X, const float* __restrict__ W,
               const float* __restrict__ b, float* __restrict__ Z, float* __restrict__ H, int act) {
  __shared__ float Ws[HID * HID];
  __shared__ float Xs[ROWS_PER_BLOCK * HID];
  for (int i = threadIdx.x; i < K * N; i += blockDim.x) Ws[i] = W[i];
  const int r0 = blockIdx.x * ROWS_PER_BLOCK;
  for (int i = threadIdx.x; i < ROWS_PER_BLOCK * K; i += blockDim.x) {
    const int r = r0 + i / K;
    Xs[i] = r < rows ? X[static_cast<int64_t>(r) * K + i % K] : 0.0f;
  }
  __syncthreads();
  for (int o = threadIdx.x; o < ROWS_PER_BLOCK * N; o += blockDim.x) {
    const int rl = o / N, j = o % N;
    const int r = r0 + rl;
    if (r >= rows) continue;
    float acc = b[j];
    for (int k = 0; k < K; ++k) acc += Xs[rl * K + k] * Ws[k * N + j];
    if (Z) Z[static_cast<int64_t>(r) * N + j] = acc;
    H[static_cast<int64_t>(r) * N + j] = act ? gelu_f(acc) : acc;
  }
}

// Dp[r][k] = (sum_j D[r][j] W[k][j]) * gelu'(Zp[r][k])
__global__ void __launch_bounds__(256)
    linear_bwd_data(int rows, int K, int N, const float* __restrict__ D, const float* __restrict__ W,
                    const float* __restrict__ Zp, float* __restrict__ Dp) {
  __shared__ float Ws[HID * HID];
  __shared__ float Ds[ROWS_PER_BLOCK * HID];
  for (int i = threadIdx.x; i < K * N; i += blockDim.x) Ws[i] = W[i];
  const int r0 = blockIdx.x * ROWS_PER_BLOCK;
  for (int i = threadIdx.x; i < ROWS_PER_BLOCK * N; i += blockDim.x) {
    const int r = r0 + i / N;
    Ds[i] = r < rows ? D[static_cast<int64_t>(r) * N + i % N] : 0.0f;
  }
  __syncthreads();
  for (int o = threadIdx.x; o < ROWS_PER_BLOCK * K; o += blockDim.x) {
    const int rl = o / K, k = o % K;
    const int r = r0 + rl;
    if (r >= rows) continue;
    float acc = 0.0f;
    for (int j = 0; j < N; ++j) acc += Ds[rl * N + j] * Ws[k * N + j];
    Dp[static_cast<int64_t>(r) * K + k] = acc * gelu_df(Zp[static_cast<int64_t>(r) * K + k]);
  }
}

// gW[k][j] += sum_r X[r][k] D[r][j]; gb[j] += sum_r D[r][j]  (rows of this block)
__global__ void __launch_bounds__(256)
    linear_bwd_weight(int rows, int K, int N, const float* __restrict__ X, const float* __restrict__ D,
                      float* __restrict__ gW, float* __restrict__ gb) {
  __shared__ float Xs[ROWS_PER_BLOCK * HID];
  __shared__ float Ds[ROWS_PER_BLOCK * HID];
  const int r0 = blockIdx.x * ROWS_PER_BLOCK;
  for (int i = threadIdx.x; i < ROWS_PER_BLOCK * K; i += blockDim.x) {
    const int r = r0 + i / K;
    Xs[i] = r < rows ? X[static_cast<int64_t>(r) * K + i % K] : 0.0f;
  }
  for (int i = threadIdx.x; i < ROWS_PER_BLOCK * N; i += blockDim.x) {
    const int r = r0 + i / N;
    Ds[i] = r < rows ? D[static_cast<int64_t>(r) * N + i % N] : 0.0f;
  }
  __syncthreads();
  for (int o = threadIdx.x; o < (K + 1) * N; o += blockDim.x) {
    const int k = o / N, j = o % N;
    float acc = 0.0f;
    if (k < K) {
      for (int rl = 0; rl < ROWS_PER_BLOCK; ++rl) acc += Xs[rl * K + k] * Ds[rl * N + j];
      atomicAdd(&gW[k * N + j], acc);
    } else {
      for (int rl = 0; rl < ROWS_PER_BLOCK; ++rl) acc += Ds[rl * N + j];
      atomicAdd(&gb[j], acc);
    }
  }
}

// D = 2 (Y - T) / count; loss partial sums of (Y - T)^2
__global__ void mse_grad(int64_t n, float inv_count, const float* __restrict__ Y, const float* __restrict__ T,
                         float* __restrict__ D, float* __restrict__ loss_acc) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float d = Y[i] - T[i];
    D[i] = 2.0f * d * inv_count;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss_acc) atomicAdd(loss_acc, red[0] * inv_count);
}

__global__ void adam_step(int n, float lr, float b1, float b2, float eps, float c1, float c2,
                          float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                          float* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void zero_f(int64_t n, float* __restrict__ x) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    x[i] = 0.0f;
}

__global__ void gather_rows_k(int nr, int nin, int nq, const int64_t* __restrict__ idx, const float* __restrict__ X,
                              const float* __restrict__ T, float* __restrict__ xb, float* __restrict__ tb) {
  const int r = blockIdx.x;
  if (r >= nr) return;
  const int64_t src = idx[r];
  for (int i = threadIdx.x; i < nin; i += blockDim.x) xb[static_cast<int64_t>(r) * nin + i] = X[src * nin + i];
  for (int i = threadIdx.x; i < nq; i += blockDim.x) tb[static_cast<int64_t>(r) * nq + i] = T[src * nq + i];
}

// rows of the data set: pair p, coarse cell c -> X (b / s at the nodes,
// centre), T (exact / s at the nodes)
__global__ void build_rows(int n_pairs, int n_cells, int nq, int n0, const double* __restrict__ B,
                           const double* __restrict__ Xs, const int32_t* __restrict__ node_dof,
                           const float* __restrict__ centre, float* __restrict__ X, float* __restrict__ T) {
  const int64_t row = blockIdx.x;
  if (row >= static_cast<int64_t>(n_pairs) * n_cells) return;
  const int p = static_cast<int>(row / n_cells), c = static_cast<int>(row % n_cells);
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n0; i += blockDim.x) s += B[static_cast<int64_t>(p) * n0 + i] * B[static_cast<int64_t>(p) * n0 + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double inv = red[0] > 0 ? 1.0 / sqrt(red[0]) : 0.0;
  const int nin = nq + 3;
  for (int q = threadIdx.x; q < nq; q += blockDim.x) {
    const int d = node_dof[c * nq + q];
    X[row * nin + q] = d < 0 ? 0.0f : static_cast<float>(B[static_cast<int64_t>(p) * n0 + d] * inv);
    T[row * nq + q] = d < 0 ? 0.0f : static_cast<float>(Xs[static_cast<int64_t>(p) * n0 + d] * inv);
  }
  if (threadIdx.x < 3) X[row * nin + nq + threadIdx.x] = centre[3 * c + threadIdx.x];
}

// out[p][i] = sum_j A[i][j] in[p][j]   (FP64, one block per (pair, 64 rows))
__global__ void __launch_bounds__(256)
    batched_dense_mv(int n_pairs, int n0, const double* __restrict__ A, const double* __restrict__ in,
                     double* __restrict__ out) {
  const int p = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + threadIdx.x / 64;
  if (row >= n0) return;
  double s = 0.0;
  for (int j = lane; j < n0; j += 64) s += A[static_cast<int64_t>(row) * n0 + j] * in[static_cast<int64_t>(p) * n0 + j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) out[static_cast<int64_t>(p) * n0 + row] = s;
}

// Coarse solve by the network, step 1: one block of 64 threads per coarse
// cell evaluates the MLP and adds its averaged nodal outputs to y (= work
// + n0, zeroed beforehand); every block recomputes s = ||b0||_2.
template <typename S>
__global__ void __launch_bounds__(64)
    net_infer_cells(int n0, int nq, const float* __restrict__ theta, const int32_t* __restrict__ node_dof,
                    const float* __restrict__ inv_val, const float* __restrict__ centre, const S* __restrict__ b,
                    double* __restrict__ work) {
  __shared__ double red[64];
  __shared__ float xin[HID];
  __shared__ float h1[HID];
  __shared__ float h2[HID];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n0; i += 64) {
    const double v = load_as<double>(b[i]);
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 32; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double nb = sqrt(red[0]);
  if (nb == 0.0) return;
  const float inv = static_cast<float>(1.0 / nb);
  const int nin = nq + 3;
  const float* W1 = theta;
  const float* b1 = W1 + nin * HID;
  const float* W2 = b1 + HID;
  const float* b2 = W2 + HID * HID;
  const float* W3 = b2 + HID;
  const float* b3 = W3 + HID * nq;
  if (threadIdx.x < nq) {
    const int d = node_dof[c * nq + threadIdx.x];
    xin[threadIdx.x] = d < 0 ? 0.0f : static_cast<float>(load_as<double>(b[d])) * inv;
  } else if (threadIdx.x < nin) {
    xin[threadIdx.x] = centre[3 * c + threadIdx.x - nq];
  }
  __syncthreads();
  float acc = b1[threadIdx.x];
  for (int q = 0; q < nin; ++q) acc += xin[q] * W1[q * HID + threadIdx.x];
  h1[threadIdx.x] = gelu_f(acc);
  __syncthreads();
  acc = b2[threadIdx.x];
  for (int k = 0; k < HID; ++k) acc += h1[k] * W2[k * HID + threadIdx.x];
  h2[threadIdx.x] = gelu_f(acc);
  __syncthreads();
  if (threadIdx.x < nq) {
    acc = b3[threadIdx.x];
    for (int k = 0; k < HID; ++k) acc += h2[k] * W3[k * nq + threadIdx.x];
    const int d = node_dof[c * nq + threadIdx.x];
    if (d >= 0) atomicAdd(&work[n0 + d], static_cast<double>(acc) * nb * inv_val[d]);
  }
}

// Step 2: the exact coarse operator checks the prediction y; if
// ||b0 - A0 y|| > tau ||b0|| the exact solution A0^{-1} b0 is used instead.
// Three kernels, all on the stream (no host synchronisation):
//  net_resid: one wavefront per row i, r_i = b_i - (A0 y)_i read along the
//    row (adjacent lanes, adjacent entries); per block the sums of r_i^2 and
//    b_i^2 into partial[2 block + {0, 1}];
//  net_decide (one block): the two norms from the partials in block order,
//    the decision (flag: 0 accept, 1 reject, 2 zero right-hand side) and the
//    counters;
//  net_apply: one wavefront per row, x_i = y_i (accept), 0, or
//    (A0^{-1} b0)_i (reject; the inverse is read only then).
constexpr int NET_ROWS = 4;  // rows (wavefronts) per block of the dense kernels

inline unsigned net_row_blocks(int n0) { return static_cast<unsigned>((n0 + NET_ROWS - 1) / NET_ROWS); }

template <typename S>
__global__ void __launch_bounds__(64 * NET_ROWS)
    net_resid(int n0, const double* __restrict__ A, const S* __restrict__ b, const double* __restrict__ y,
              double* __restrict__ partial) {
  __shared__ double red[2 * NET_ROWS];
  const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
  const int row = blockIdx.x * NET_ROWS + w;
  double rr = 0.0, bb = 0.0;
  if (row < n0) {
    double s = 0.0;
    for (int j = lane; j < n0; j += 64) s += A[static_cast<int64_t>(row) * n0 + j] * y[j];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    const double bi = load_as<double>(b[row]);
    const double r = bi - s;
    rr = r * r;
    bb = bi * bi;
  }
  if (lane == 0) {
    red[2 * w] = rr;
    red[2 * w + 1] = bb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int q = 0; q < NET_ROWS; ++q) {
      a += red[2 * q];
      c += red[2 * q + 1];
    }
    partial[2 * blockIdx.x] = a;
    partial[2 * blockIdx.x + 1] = c;
  }
}

__global__ void __launch_bounds__(256)
    net_decide(int n_blocks, double tau, const double* __restrict__ partial, double* __restrict__ flag,
               int* __restrict__ counters, double* __restrict__ relsum) {
  __shared__ double ra[256], rb[256];
  double a = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < n_blocks; i += 256) {
    a += partial[2 * i];
    c += partial[2 * i + 1];
  }
  ra[threadIdx.x] = a;
  rb[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      ra[threadIdx.x] += ra[threadIdx.x + w];
      rb[threadIdx.x] += rb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nb = sqrt(rb[0]);
    if (nb == 0.0) {
      flag[0] = 2.0;
      return;
    }
    const double rel = sqrt(ra[0]) / nb;
    const bool accept = rel <= tau;
    flag[0] = accept ? 0.0 : 1.0;
    atomicAdd(&counters[accept ? 0 : 1], 1);
    atomicAdd(relsum, rel);
  }
}

// mode 2 (no coarse correction) writes zeros without reading the flag
template <typename S>
__global__ void __launch_bounds__(64 * NET_ROWS)
    net_apply(int n0, int mode, const double* __restrict__ Ainv, const S* __restrict__ b,
              const double* __restrict__ y, const double* __restrict__ flag, S* __restrict__ x) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * NET_ROWS + threadIdx.x / 64;
  if (row >= n0) return;
  const double f = mode == 2 ? 2.0 : flag[0];
  if (f == 1.0) {
    double v = 0.0;
    for (int j = lane; j < n0; j += 64) v += Ainv[static_cast<int64_t>(row) * n0 + j] * load_as<double>(b[j]);
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) x[row] = store_as<S>(v);
  } else if (lane == 0) {
    x[row] = store_as<S>(f == 0.0 ? y[row] : 0.0);
  }
}

unsigned blocks_for(int64_t n, int per = 256) {
  int64_t b = (n + per - 1) / per;
  return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(b, 1 << 20)));
}

}  // namespace

int net_n_params(int nq) { return (nq + 3) * HID + HID + HID * HID + HID + HID * nq + nq; }

// The kernels stage one row of inputs (nq + 3 values) and the weight blocks
// in arrays of the hidden width, and run one thread per output node.
bool net_supported(int k) { return (k + 1) * (k + 1) * (k + 1) + 3 <= HID; }

void net_setup(Context& ctx, const LevelDofs& L0) {
  NetState& N = ctx.net;
  MFMG_REQUIRE(net_supported(L0.k), MFMG_ERR_UNSUPPORTED, "coarse degree too high for the network width");
  N.nq = (L0.k + 1) * (L0.k + 1) * (L0.k + 1);
  N.n_cells = static_cast<int>(L0.n_cells);
  N.n0 = static_cast<int>(L0.n_dofs);
  const int k = L0.k, n = k + 1;
  std::vector<int32_t> nd(static_cast<size_t>(N.n_cells) * N.nq, -1);
  std::vector<float> val(N.n0, 0.0f), ctr(3 * N.n_cells);
  for (int64_t c = 0; c < L0.n_cells; ++c) {
    MFMG_REQUIRE(!mask_hanging(L0.mask[c]), MFMG_ERR_UNSUPPORTED, "coarse level with hanging nodes");
    for (int cc = 0; cc < n; ++cc)
      for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
          const int s = node_slot(a, b, cc, k);
          const int32_t e = L0.ent[s * L0.n_cells + c];
          const int q = a + n * b + n * n * cc;
          nd[c * N.nq + q] = e < 0 ? -1 : e + node_offset(a, b, cc, k);
          if (e >= 0) val[e + node_offset(a, b, cc, k)] += 1.0f;
        }
    const double h = L0.h0 * std::ldexp(1.0, -L0.cells[c].level);
    ctr[3 * c + 0] = static_cast<float>(ctx.meshes[0].lo + (L0.cells[c].i + 0.5) * h);
    ctr[3 * c + 1] = static_cast<float>(ctx.meshes[0].lo + (L0.cells[c].j + 0.5) * h);
    ctr[3 * c + 2] = static_cast<float>(ctx.meshes[0].lo + (L0.cells[c].k + 0.5) * h);
  }
  for (auto& v : val) v = v > 0 ? 1.0f / v : 0.0f;
  N.node_dof.upload(nd);
  N.inv_val.upload(val);
  N.centre.upload(ctr);
  N.n_params = net_n_params(N.nq);
  N.params.alloc(N.n_params);
  std::vector<float> zeros(N.n_params, 0.0f);
  MFMG_HIP(hipMemcpy(N.params.ptr, zeros.data(), N.n_params * 4, hipMemcpyHostToDevice));
  // y (n0), a spare n0, the decision flag (8 slots) and 2 partial sums per
  // block of the dense check
  N.work.alloc(2 * static_cast<size_t>(N.n0) + 8 + 2 * static_cast<size_t>(net_row_blocks(N.n0)));
  N.counters.alloc(2);
  MFMG_HIP(hipMemset(N.counters.ptr, 0, 8));
  N.relsum.alloc(1);
  MFMG_HIP(hipMemset(N.relsum.ptr, 0, 8));
}

void net_init_params(Context& ctx, uint64_t seed) {
  NetState& N = ctx.net;
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<float> p(N.n_params, 0.0f);
  const int sizes[4] = {N.nq + 3, HID, HID, N.nq};
  size_t off = 0;
  for (int l = 0; l < 3; ++l) {
    const int a = sizes[l], b = sizes[l + 1];
    for (int i = 0; i < a * b; ++i) p[off + i] = static_cast<float>(nd(rng) * std::sqrt(2.0 / a));
    off += a * b + b;
  }
  MFMG_HIP(hipMemcpy(N.params.ptr, p.data(), N.n_params * 4, hipMemcpyHostToDevice));
}

// loss (accumulated into N.lossbuf) and gradient over `rows` rows with the
// current parameters; asynchronous
static void net_loss_grad_async(Context& ctx, int rows, const float* X, const float* T, float* grad,
                                hipStream_t s) {
  NetState& N = ctx.net;
  const int nin = N.nq + 3, nq = N.nq;
  auto ensure = [&](DeviceArray<float>& a, size_t n) {
    if (a.n < n) a.alloc(n);
  };
  ensure(N.z1, static_cast<size_t>(rows) * HID);
  ensure(N.h1, static_cast<size_t>(rows) * HID);
  ensure(N.z2, static_cast<size_t>(rows) * HID);
  ensure(N.h2, static_cast<size_t>(rows) * HID);
  ensure(N.y, static_cast<size_t>(rows) * nq);
  ensure(N.d3, static_cast<size_t>(rows) * nq);
  ensure(N.d2, static_cast<size_t>(rows) * HID);
  ensure(N.d1, static_cast<size_t>(rows) * HID);
  ensure(N.lossbuf, 1);
  const float* p = N.params.ptr;
  const float *W1 = p, *b1 = W1 + nin * HID, *W2 = b1 + HID, *b2 = W2 + HID * HID, *W3 = b2 + HID,
              *b3 = W3 + HID * nq;
  float *gW1 = grad, *gb1 = gW1 + nin * HID, *gW2 = gb1 + HID, *gb2 = gW2 + HID * HID, *gW3 = gb2 + HID,
        *gb3 = gW3 + HID * nq;
  const unsigned g = static_cast<unsigned>((rows + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK);
  zero_f<<<blocks_for(N.n_params), 256, 0, s>>>(N.n_params, grad);
  zero_f<<<1, 256, 0, s>>>(1, N.lossbuf.ptr);
  linear_fwd<<<g, 256, 0, s>>>(rows, nin, HID, X, W1, b1, N.z1.ptr, N.h1.ptr, 1);
  linear_fwd<<<g, 256, 0, s>>>(rows, HID, HID, N.h1.ptr, W2, b2, N.z2.ptr, N.h2.ptr, 1);
  linear_fwd<<<g, 256, 0, s>>>(rows, HID, nq, N.h2.ptr, W3, b3, nullptr, N.y.ptr, 0);
  const int64_t ny = static_cast<int64_t>(rows) * nq;
  mse_grad<<<blocks_for(ny), 256, 0, s>>>(ny, 1.0f / static_cast<float>(ny), N.y.ptr, T, N.d3.ptr, N.lossbuf.ptr);
  linear_bwd_weight<<<g, 256, 0, s>>>(rows, HID, nq, N.h2.ptr, N.d3.ptr, gW3, gb3);
  linear_bwd_data<<<g, 256, 0, s>>>(rows, HID, nq, N.d3.ptr, W3, N.z2.ptr, N.d2.ptr);
  linear_bwd_weight<<<g, 256, 0, s>>>(rows, HID, HID, N.h1.ptr, N.d2.ptr, gW2, gb2);
  linear_bwd_data<<<g, 256, 0, s>>>(rows, HID, HID, N.d2.ptr, W2, N.z1.ptr, N.d1.ptr);
  linear_bwd_weight<<<g, 256, 0, s>>>(rows, nin, HID, X, N.d1.ptr, gW1, gb1);
  check_launch();
}

float net_loss_grad(Context& ctx, int rows, const float* X, const float* T, float* grad, hipStream_t s) {
  net_loss_grad_async(ctx, rows, X, T, grad, s);
  float loss = 0.0f;
  MFMG_HIP(hipMemcpyAsync(&loss, ctx.net.lossbuf.ptr, 4, hipMemcpyDeviceToHost, s));
  MFMG_HIP(hipStreamSynchronize(s));
  return loss;
}

void net_train(Context& ctx, const mfmg_net_train_desc& d, float* history, hipStream_t s) {
  NetState& N = ctx.net;
  MFMG_REQUIRE(N.rec_count > 0, MFMG_ERR_INVALID_ARG, "no recorded coarse right-hand sides");
  const int P = N.rec_count, n0 = N.n0, nq = N.nq, nin = nq + 3;
  // exact coarse solutions of the recorded right-hand sides
  DeviceArray<double> xs(static_cast<size_t>(P) * n0);
  batched_dense_mv<<<dim3((n0 + 3) / 4, P), 256, 0, s>>>(P, n0, ctx.coarse_inv64.ptr, N.record.ptr, xs.ptr);
  check_launch();
  const int64_t rows = static_cast<int64_t>(P) * N.n_cells;
  MFMG_REQUIRE(rows < (1ll << 31), MFMG_ERR_UNSUPPORTED, "too many training rows");
  N.X.alloc(rows * nin);
  N.T.alloc(rows * nq);
  build_rows<<<static_cast<unsigned>(rows), 256, 0, s>>>(P, N.n_cells, nq, n0, N.record.ptr, xs.ptr, N.node_dof.ptr,
                                                         N.centre.ptr, N.X.ptr, N.T.ptr);
  check_launch();
  if (d.init_seed != 0) net_init_params(ctx, d.init_seed);
  const int B = d.batch_rows > 0 ? d.batch_rows : 4096;
  DeviceArray<float> grad(N.n_params), m(N.n_params), v(N.n_params), xb(static_cast<size_t>(B) * nin),
      tb(static_cast<size_t>(B) * nq);
  zero_f<<<blocks_for(N.n_params), 256, 0, s>>>(N.n_params, m.ptr);
  zero_f<<<blocks_for(N.n_params), 256, 0, s>>>(N.n_params, v.ptr);
  std::mt19937_64 rng(d.shuffle_seed);
  std::vector<int64_t> perm(rows);
  std::iota(perm.begin(), perm.end(), 0);
  const float lr = static_cast<float>(d.lr > 0 ? d.lr : 1e-3);
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  int64_t t = 0;
  DeviceArray<int64_t> dperm(rows);
  for (int e = 0; e < d.epochs; ++e) {
    std::shuffle(perm.begin(), perm.end(), rng);
    MFMG_HIP(hipMemcpyAsync(dperm.ptr, perm.data(), rows * 8, hipMemcpyHostToDevice, s));
    double acc = 0.0;
    int nb = 0;
    for (int64_t r0 = 0; r0 < rows; r0 += B) {
      const int nr = static_cast<int>(std::min<int64_t>(B, rows - r0));
      gather_rows_k<<<static_cast<unsigned>(nr), 64, 0, s>>>(nr, nin, nq, dperm.ptr + r0, N.X.ptr, N.T.ptr, xb.ptr,
                                                              tb.ptr);
      net_loss_grad_async(ctx, nr, xb.ptr, tb.ptr, grad.ptr, s);
      ++t;
      const float c1 = 1.0f - std::pow(b1, static_cast<float>(t)), c2 = 1.0f - std::pow(b2, static_cast<float>(t));
      adam_step<<<blocks_for(N.n_params), 256, 0, s>>>(N.n_params, lr, b1, b2, eps, c1, c2, N.params.ptr, grad.ptr,
                                                        m.ptr, v.ptr);
      check_launch();
      ++nb;
    }
    // epoch loss on the whole data set (same rows, current parameters)
    for (int64_t r0 = 0; r0 < rows; r0 += B) {
      const int nr = static_cast<int>(std::min<int64_t>(B, rows - r0));
      acc += static_cast<double>(net_loss_grad(ctx, nr, N.X.ptr + r0 * nin, N.T.ptr + r0 * nq, grad.ptr, s)) * nr;
    }
    if (history) history[e] = static_cast<float>(acc / rows);
    (void)nb;
  }
}

template <typename S>
static void net_coarse_solve_t(Context& ctx, S* x, const S* b, hipStream_t s) {
  NetState& N = ctx.net;
  const int mode = N.mode == MFMG_COARSE_ZERO ? 2 : 1;
  if (mode == 1) {
    // y = work[n0 .. 2 n0) (doubles) starts at zero
    zero_f<<<1, 256, 0, s>>>(2 * static_cast<int64_t>(N.n0), reinterpret_cast<float*>(N.work.ptr + N.n0));
    net_infer_cells<S><<<N.n_cells, 64, 0, s>>>(N.n0, N.nq, N.params.ptr, N.node_dof.ptr, N.inv_val.ptr,
                                                 N.centre.ptr, b, N.work.ptr);
  }
  const unsigned nbk = net_row_blocks(N.n0);
  double* flag = N.work.ptr + 2 * static_cast<int64_t>(N.n0);
  double* partial = flag + 8;
  if (mode == 1) {
    net_resid<S><<<nbk, 64 * NET_ROWS, 0, s>>>(N.n0, ctx.coarse_A64.ptr, b, N.work.ptr + N.n0, partial);
    net_decide<<<1, 256, 0, s>>>(static_cast<int>(nbk), N.tau, partial, flag, N.counters.ptr, N.relsum.ptr);
  }
  net_apply<S><<<nbk, 64 * NET_ROWS, 0, s>>>(N.n0, mode, ctx.coarse_inv64.ptr, b, N.work.ptr + N.n0, flag, x);
  check_launch();
}

template <typename S>
static void net_predict_t(Context& ctx, S* y, const S* b, hipStream_t s) {
  NetState& N = ctx.net;
  zero_f<<<1, 256, 0, s>>>(2 * static_cast<int64_t>(N.n0), reinterpret_cast<float*>(N.work.ptr + N.n0));
  net_infer_cells<S><<<N.n_cells, 64, 0, s>>>(N.n0, N.nq, N.params.ptr, N.node_dof.ptr, N.inv_val.ptr,
                                               N.centre.ptr, b, N.work.ptr);
  check_launch();
  launch_cast_from_f64(dtype_of<S>(), N.n0, N.work.ptr + N.n0, y, s);
}

void net_predict(Context& ctx, int dtype, void* y, const void* b, hipStream_t s) {
  switch (dtype) {
    case MFMG_F64: net_predict_t<double>(ctx, static_cast<double*>(y), static_cast<const double*>(b), s); break;
    case MFMG_F32: net_predict_t<float>(ctx, static_cast<float*>(y), static_cast<const float*>(b), s); break;
    case MFMG_BF16: net_predict_t<bf16>(ctx, static_cast<bf16*>(y), static_cast<const bf16*>(b), s); break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "dtype");
  }
}

void net_coarse_solve(Context& ctx, int dtype, void* x, const void* b, hipStream_t s) {
  switch (dtype) {
    case MFMG_F64: net_coarse_solve_t<double>(ctx, static_cast<double*>(x), static_cast<const double*>(b), s); break;
    case MFMG_F32: net_coarse_solve_t<float>(ctx, static_cast<float*>(x), static_cast<const float*>(b), s); break;
    case MFMG_BF16: net_coarse_solve_t<bf16>(ctx, static_cast<bf16*>(x), static_cast<const bf16*>(b), s); break;
    default: throw Error(MFMG_ERR_UNSUPPORTED, "dtype");
  }
}

}  // namespace mfmg
