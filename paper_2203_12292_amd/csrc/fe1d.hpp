// One-dimensional Lagrange element tables (host side, double precision).
//
// The tensor-product Q_k element is fully described by 1D quantities on
// [0, 1]: the Gauss-Lobatto nodes xi_0..xi_k, the (k+1)-point Gauss rule,
// the 1D mass matrix M and stiffness matrix K (both integrated exactly by the
// Gauss rule), the interpolation of a coarse interval onto its two halves
// (hanging-node constraints, Section 3.1) and the 1D prolongation matrices of
// the transfer categories (Section 3.5).
#pragma once

#include <cmath>
#include <vector>

namespace mfmg {

// Legendre P_n(x) and P_n'(x) on [-1, 1] by the three-term recurrence.
inline void legendre(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { p = 1.0; dp = 0.0; return; }
  for (int m = 2; m <= n; ++m) {
    double p2 = ((2.0 * m - 1.0) * x * p1 - (m - 1.0) * p0) / m;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  // (1 - x^2) P_n' = n (P_{n-1} - x P_n)
  dp = (std::fabs(1.0 - x * x) < 1e-300) ? 0.0 : n * (p0 - x * p1) / (1.0 - x * x);
}

// Gauss-Lobatto-Legendre nodes of degree k mapped to [0, 1]: the end points
// and the roots of P_k', found by Newton's method on P_k' using the Legendre
// differential equation for P_k''.
inline std::vector<double> gll_nodes(int k) {
  std::vector<double> x(k + 1);
  x[0] = -1.0;
  x[k] = 1.0;
  for (int j = 1; j < k; ++j) {
    double t = -std::cos(M_PI * j / k);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(k, t, p, dp);
      double d2p = (2.0 * t * dp - k * (k + 1.0) * p) / (1.0 - t * t);
      double step = dp / d2p;
      t -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    x[j] = t;
  }
  std::vector<double> r(k + 1);
  for (int j = 0; j <= k; ++j) {
    double s = 0.5 * (x[j] - x[k - j]);  // exact symmetry about the centre
    r[j] = 0.5 * (s + 1.0);
  }
  return r;
}

// n-point Gauss-Legendre rule on [0, 1] (Newton on P_n).
inline void gauss_rule(int n, std::vector<double>& pts, std::vector<double>& wts) {
  std::vector<double> x(n), w(n);
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double p = 0, dp = 0;
    for (int it = 0; it < 100; ++it) {
      legendre(n, t, p, dp);
      double step = p / dp;
      t -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    legendre(n, t, p, dp);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
  pts.assign(n, 0.0);
  wts.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {  // ascending order, symmetric
    int j = n - 1 - i;
    double s = 0.5 * (x[j] - x[i]);
    pts[i] = 0.5 * (s + 1.0);
    wts[i] = 0.25 * (w[i] + w[j]);
  }
}

// Lagrange basis on `nodes`: value of l_j at t.
inline double lagrange(const std::vector<double>& nodes, int j, double t) {
  double v = 1.0;
  for (size_t m = 0; m < nodes.size(); ++m)
    if ((int)m != j) v *= (t - nodes[m]) / (nodes[j] - nodes[m]);
  return v;
}

inline double lagrange_deriv(const std::vector<double>& nodes, int j, double t) {
  double s = 0.0;
  for (size_t m = 0; m < nodes.size(); ++m) {
    if ((int)m == j) continue;
    double term = 1.0 / (nodes[j] - nodes[m]);
    for (size_t q = 0; q < nodes.size(); ++q)
      if ((int)q != j && q != m) term *= (t - nodes[q]) / (nodes[j] - nodes[q]);
    s += term;
  }
  return s;
}

struct Tables1D {
  int k = 0, n = 0;
  std::vector<double> nodes, qp, qw;
  std::vector<double> M, K;     // n x n, row-major
  std::vector<double> S;        // S[q*n+i] = l_i(qp_q)
  std::vector<double> H[2];     // H[s][i*n+j] = l_j((s + xi_i)/2)
  std::vector<double> T;        // (2k+1) x n: coarse node j -> node I of the two halves

  explicit Tables1D(int deg = 1) { build(deg); }

  void build(int deg) {
    k = deg;
    n = deg + 1;
    nodes = gll_nodes(k);
    gauss_rule(n, qp, qw);
    M.assign(n * n, 0.0);
    K.assign(n * n, 0.0);
    S.assign(n * n, 0.0);
    for (int q = 0; q < n; ++q)
      for (int i = 0; i < n; ++i) S[q * n + i] = lagrange(nodes, i, qp[q]);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double m = 0, kk = 0;
        for (int q = 0; q < n; ++q) {
          m += qw[q] * lagrange(nodes, i, qp[q]) * lagrange(nodes, j, qp[q]);
          kk += qw[q] * lagrange_deriv(nodes, i, qp[q]) * lagrange_deriv(nodes, j, qp[q]);
        }
        M[i * n + j] = m;
        K[i * n + j] = kk;
      }
    for (int s = 0; s < 2; ++s) {
      H[s].assign(n * n, 0.0);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) H[s][i * n + j] = clean(lagrange(nodes, j, 0.5 * (s + nodes[i])));
    }
    int m = 2 * k + 1;
    T.assign(m * n, 0.0);
    for (int I = 0; I < m; ++I) {
      double t = (I <= k) ? 0.5 * nodes[I] : 0.5 * (1.0 + nodes[I - k]);
      for (int j = 0; j < n; ++j) T[I * n + j] = clean(lagrange(nodes, j, t));
    }
  }

  // exact zeros/ones where the point is a node
  static double clean(double v) {
    if (std::fabs(v) < 1e-14) return 0.0;
    if (std::fabs(v - 1.0) < 1e-14) return 1.0;
    return v;
  }
};

// Polynomial-coarsening prolongation: coarse degree kc basis at fine nodes.
inline std::vector<double> p_transfer_matrix(int kf, int kc) {
  std::vector<double> nf = gll_nodes(kf), nc = gll_nodes(kc);
  std::vector<double> T((kf + 1) * (kc + 1));
  for (int i = 0; i <= kf; ++i)
    for (int j = 0; j <= kc; ++j) T[i * (kc + 1) + j] = Tables1D::clean(lagrange(nc, j, nf[i]));
  return T;
}

// h and p coarsening in one step: the coarse degree-kc basis on [0,1]
// evaluated at the degree-kf nodes of the two halves (2 kf + 1 points, the
// shared middle node once), row-major (2 kf + 1) x (kc + 1)
inline std::vector<double> hp_transfer_matrix(int kf, int kc) {
  std::vector<double> nf = gll_nodes(kf), nc = gll_nodes(kc);
  const int m = 2 * kf + 1;
  std::vector<double> T(m * (kc + 1));
  for (int I = 0; I < m; ++I) {
    const double t = (I <= kf) ? 0.5 * nf[I] : 0.5 * (1.0 + nf[I - kf]);
    for (int j = 0; j <= kc; ++j) T[I * (kc + 1) + j] = Tables1D::clean(lagrange(nc, j, t));
  }
  return T;
}

}  // namespace mfmg
