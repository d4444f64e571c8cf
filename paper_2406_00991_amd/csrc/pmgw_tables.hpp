// Host-side constant tables of the p-multigrid hierarchy (Chebyshev-Gauss-Lobatto nodes,
// the collocation derivative in sigma, restriction and prolongation between orders), shared by
// the 2D and 3D libraries.
#pragma once
#include <cmath>
#include <vector>

namespace pmgw_tables {

// ----------------------------------------------------------------------------- constant tables
// Chebyshev-Gauss-Lobatto nodes xi_j = cos(j pi / M); sigma = (1 + xi)/2.
inline std::vector<double> cgl_sigma(int M) {
  std::vector<double> s(M + 1);
  for (int j = 0; j <= M; ++j) s[j] = 0.5 * (1.0 + std::cos(M_PI * j / M));
  s[M] = 0.0;
  s[0] = 1.0;
  return s;
}

// d/dsigma on the CGL nodes: twice the closed-form Chebyshev collocation derivative in xi,
// with node differences written as products of sines and a negative-sum diagonal.
inline std::vector<double> dsigma(int M) {
  const int n = M + 1;
  std::vector<double> D(n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double rs = 0.0;
    for (int l = 0; l < n; ++l) {
      if (l == j) continue;
      const double cj = (j == 0 || j == M) ? 2.0 : 1.0;
      const double cl = (l == 0 || l == M) ? 2.0 : 1.0;
      const double diff = 2.0 * std::sin((j + l) * M_PI / (2.0 * M)) *
                          std::sin((l - j) * M_PI / (2.0 * M));
      const double v = (cj / cl) * (((j + l) & 1) ? -1.0 : 1.0) / diff;
      D[j * n + l] = 2.0 * v;
      rs += 2.0 * v;
    }
    D[j * n + j] = -rs;
  }
  return D;
}

// T_m(cos(theta)) = cos(m theta).
inline double cheb_T(int m, double theta) { return std::cos(m * theta); }

// Restriction fine order Mf -> Mc = Mf/2: nodal values -> Chebyshev coefficients, keep m <= Mc,
// evaluate at the coarse nodes; surface and bed rows are injected. [(Mc+1)][(Mf+1)].
// B = A^T for a row-major rows x cols matrix A.
inline std::vector<double> transpose(const std::vector<double>& A, int rows, int cols) {
  std::vector<double> B((size_t)rows * cols);
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) B[(size_t)c * rows + r] = A[(size_t)r * cols + c];
  return B;
}

inline std::vector<double> restriction(int Mf) {
  const int Mc = Mf / 2, nf = Mf + 1, nc = Mc + 1;
  std::vector<double> R(nc * nf, 0.0);
  for (int jc = 0; jc < nc; ++jc) {
    const double th = M_PI * jc / Mc;
    for (int l = 0; l < nf; ++l) {
      const double cl = (l == 0 || l == Mf) ? 2.0 : 1.0;
      double s = 0.0;
      for (int m = 0; m <= Mc; ++m) {
        const double cm = (m == 0 || m == Mf) ? 2.0 : 1.0;
        s += cheb_T(m, th) * (2.0 / (Mf * cm * cl)) * std::cos(M_PI * m * l / Mf);
      }
      R[jc * nf + l] = s;
    }
  }
  for (int l = 0; l < nf; ++l) {
    R[0 * nf + l] = (l == 0) ? 1.0 : 0.0;
    R[Mc * nf + l] = (l == Mf) ? 1.0 : 0.0;
  }
  return R;
}

// Prolongation Mc -> Mf: the coarse interpolating polynomial evaluated at the fine nodes.
inline std::vector<double> prolongation(int Mf) {
  const int Mc = Mf / 2, nf = Mf + 1, nc = Mc + 1;
  std::vector<double> P(nf * nc, 0.0);
  for (int j = 0; j < nf; ++j) {
    const double th = M_PI * j / Mf;
    for (int c = 0; c < nc; ++c) {
      const double cc = (c == 0 || c == Mc) ? 2.0 : 1.0;
      double s = 0.0;
      for (int m = 0; m <= Mc; ++m) {
        const double cm = (m == 0 || m == Mc) ? 2.0 : 1.0;
        s += cheb_T(m, th) * (2.0 / (Mc * cm * cc)) * std::cos(M_PI * m * c / Mc);
      }
      P[j * nc + c] = s;
    }
    if ((j & 1) == 0) {
      for (int c = 0; c < nc; ++c) P[j * nc + c] = (c == j / 2) ? 1.0 : 0.0;
    }
  }
  return P;
}

inline int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

}  // namespace pmgw_tables
