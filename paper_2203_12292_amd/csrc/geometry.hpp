// Mapped cells: the general form of the quadrature-point operation Q_e of
// Eq. (impl:mf), w_q |det J_q| J_q^{-1} J_q^{-T}, with J = dx/dxi of the
// cell map (Section 3.2), for cells that are not axis-aligned cubes.
//
// Compressed geometry.  A geometry descriptor moves the vertices of the
// coarse grid; coarse cell C becomes the trilinear image F_C of the unit cube
// through its eight moved vertices, and a cell of level l with integer
// position r inside C inherits F_e(xi) = F_C((r + xi) 2^-l) (the restriction
// of a trilinear map to a sub-box is trilinear, so the levels stay nested).
// The device holds one record of 24 numbers per coarse cell, the monomial
// coefficients of F_C,
//   F_C(t) = A0 + A1 t1 + A2 t2 + A3 t3 + A12 t1 t2 + A13 t1 t3 + A23 t2 t3
//            + A123 t1 t2 t3    (each A a 3-vector, stored [monomial][xyz]),
// and a cell finds its own map from its level and lattice position, which
// the operator has anyway: 12 bytes per cell plus 192 bytes per coarse cell.
//
// Kinds: 0 none (cubes); 1 affine, x' = M x with
// M = [[p0, p1, p2], [0, p3, p4], [0, 0, p5]]; 2 interior bump,
// x' = x + p0 s(x) (p1, p2, p3), s(x) = prod_d sin(pi (x_d - lo)/(hi - lo)),
// which leaves the boundary of [lo, hi]^3 in place.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

namespace mfmg {

struct GeoDesc {
  int kind = 0;
  double p[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

// moved position of the point x (host)
inline void geo_move(const GeoDesc& g, double lo, double hi, const double x[3], double y[3]) {
  if (g.kind == 1) {
    y[0] = g.p[0] * x[0] + g.p[1] * x[1] + g.p[2] * x[2];
    y[1] = g.p[3] * x[1] + g.p[4] * x[2];
    y[2] = g.p[5] * x[2];
  } else if (g.kind == 2) {
    const double pi = 3.14159265358979323846;
    double s = 1.0;
    for (int d = 0; d < 3; ++d) s *= std::sin(pi * (x[d] - lo) / (hi - lo));
    for (int d = 0; d < 3; ++d) y[d] = x[d] + g.p[0] * s * g.p[1 + d];
  } else {
    for (int d = 0; d < 3; ++d) y[d] = x[d];
  }
}

// [n0^3][8][3] monomial coefficients of the coarse-cell maps, coarse cell
// (I, J, K) at index I + n0 (J + n0 K)
inline std::vector<double> geometry_table(const GeoDesc& g, int n0, double lo, double hi) {
  std::vector<double> t(static_cast<size_t>(n0) * n0 * n0 * 24);
  const double h = (hi - lo) / n0;
  for (int K = 0; K < n0; ++K)
    for (int J = 0; J < n0; ++J)
      for (int I = 0; I < n0; ++I) {
        double X[8][3];
        for (int v = 0; v < 8; ++v) {
          const double x[3] = {lo + h * (I + (v & 1)), lo + h * (J + ((v >> 1) & 1)), lo + h * (K + ((v >> 2) & 1))};
          geo_move(g, lo, hi, x, X[v]);
        }
        double* A = &t[(static_cast<size_t>(I) + n0 * (J + static_cast<size_t>(n0) * K)) * 24];
        for (int d = 0; d < 3; ++d) {
          A[0 * 3 + d] = X[0][d];
          A[1 * 3 + d] = X[1][d] - X[0][d];
          A[2 * 3 + d] = X[2][d] - X[0][d];
          A[3 * 3 + d] = X[4][d] - X[0][d];
          A[4 * 3 + d] = X[3][d] - X[1][d] - X[2][d] + X[0][d];
          A[5 * 3 + d] = X[5][d] - X[1][d] - X[4][d] + X[0][d];
          A[6 * 3 + d] = X[6][d] - X[2][d] - X[4][d] + X[0][d];
          A[7 * 3 + d] = X[7][d] - X[3][d] - X[5][d] - X[6][d] + X[1][d] + X[2][d] + X[4][d] - X[0][d];
        }
      }
  return t;
}

// x = F_C(t) from the monomial coefficients A
template <typename T>
__host__ __device__ inline void geo_point(const T* __restrict__ A, T t1, T t2, T t3, T x[3]) {
  for (int d = 0; d < 3; ++d)
    x[d] = A[d] + A[3 + d] * t1 + A[6 + d] * t2 + A[9 + d] * t3 + A[12 + d] * t1 * t2 + A[15 + d] * t1 * t3 +
           A[18 + d] * t2 * t3 + A[21 + d] * t1 * t2 * t3;
}

// J[d][e] = d x_d / d t_e of F_C at t
template <typename T>
__host__ __device__ inline void geo_jacobian(const T* __restrict__ A, T t1, T t2, T t3, T J[3][3]) {
  for (int d = 0; d < 3; ++d) {
    J[d][0] = A[3 + d] + A[12 + d] * t2 + A[15 + d] * t3 + A[21 + d] * t2 * t3;
    J[d][1] = A[6 + d] + A[12 + d] * t1 + A[18 + d] * t3 + A[21 + d] * t1 * t3;
    J[d][2] = A[9 + d] + A[15 + d] * t1 + A[18 + d] * t2 + A[21 + d] * t1 * t2;
  }
}

// Metric term of one quadrature point: with the cofactor matrix C of J
// (J^{-1} = C^T / det J), w |det J| J^{-1} J^{-T} = (w / |det J|) C^T C
// (symmetric; G = {g00, g01, g02, g11, g12, g22}).
template <typename T>
__host__ __device__ inline void geo_metric(const T J[3][3], T w, T G[6], T* det_out = nullptr) {
  T C[3][3];
  C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const T det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
  const T s = w / (det < T(0) ? -det : det);
  // (C^T C)_{ij} = sum_d C[d][i] C[d][j]
  G[0] = s * (C[0][0] * C[0][0] + C[1][0] * C[1][0] + C[2][0] * C[2][0]);
  G[1] = s * (C[0][0] * C[0][1] + C[1][0] * C[1][1] + C[2][0] * C[2][1]);
  G[2] = s * (C[0][0] * C[0][2] + C[1][0] * C[1][2] + C[2][0] * C[2][2]);
  G[3] = s * (C[0][1] * C[0][1] + C[1][1] * C[1][1] + C[2][1] * C[2][1]);
  G[4] = s * (C[0][1] * C[0][2] + C[1][1] * C[1][2] + C[2][1] * C[2][2]);
  G[5] = s * (C[0][2] * C[0][2] + C[1][2] * C[1][2] + C[2][2] * C[2][2]);
  if (det_out) *det_out = det;
}

}  // namespace mfmg
