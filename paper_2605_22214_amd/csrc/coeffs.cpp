// Coefficient tables of the flux potential, computed once on the host in FP64.
//
// alpha, gamma: Eqs. alpha1/alpha2 (alpha sigma = I + gamma 1^T, alpha 1 = 0)
// are solved through the bordered matrix B = [[sigma, 1], [1^T, 0]]: its
// inverse is [[alpha, -gamma], [-gamma^T, r]].  (From B B^-1 = I the top-left
// block P satisfies sigma P + 1 q^T = I and 1^T P = 0; transposing, with P and
// sigma symmetric, P sigma = I - q 1^T and P 1 = 0, so alpha = P, gamma = -q.)
//
// Lambda (Eq. ngamma) and Theta (the system after Eq. P) are solved per index
// set on the principal sub-matrix alpha[S,S], S the complement of the three
// excluded components.  alpha is negative semidefinite with the single null
// vector 1, so every proper principal sub-matrix is negative definite.
//
// The factored tables regroup sum_j alpha_ij (mu_j + phi_j + xi_j) so that the
// bulk and stabilising parts are explicit multiples of C_i:
//  * the bulk potential on sum C = 1 is Eq. fluxwrong,
//    (12/D)[-C_i(1-3C_i+2C_i^2) + 6 sum_{j<k<l} T_{i;jkl} C_j C_k C_l];
//  * phi contributes (12/D) sum_{k<l<m} C_k C_l C_m sum_{j not in klm}
//    alpha_ij Lambda_{j;klm}, which by Eq. ngamma equals -6 T_{i;klm} for every
//    triple without i, so only triples containing i survive (Psi);
//  * in xi the Theta system cancels every C_m term with m != i for pairs
//    without i (X), and leaves an O(N) sum for pairs containing i (Z).
#include "coeffs.h"

#include <cmath>
#include <cstdio>
#include <vector>

namespace nflbm {
namespace {

// Gaussian elimination with partial pivoting on an n x n row-major matrix
// with nrhs right-hand sides (row-major n x nrhs).  Overwrites b with the
// solution.  Returns false if a pivot is below tol * (largest |entry| of A).
bool gauss_solve(std::vector<double> a, int n, std::vector<double>& b, int nrhs) {
  double scale = 0.0;
  for (double v : a) scale = std::fmax(scale, std::fabs(v));
  if (scale == 0.0) return false;
  const double tol = 1e-13 * scale;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(a[r * n + col]) > std::fabs(a[piv * n + col])) piv = r;
    if (std::fabs(a[piv * n + col]) < tol) return false;
    if (piv != col) {
      for (int c = 0; c < n; ++c) std::swap(a[piv * n + c], a[col * n + c]);
      for (int c = 0; c < nrhs; ++c) std::swap(b[piv * nrhs + c], b[col * nrhs + c]);
    }
    const double inv = 1.0 / a[col * n + col];
    for (int r = col + 1; r < n; ++r) {
      const double fct = a[r * n + col] * inv;
      if (fct == 0.0) continue;
      for (int c = col; c < n; ++c) a[r * n + c] -= fct * a[col * n + c];
      for (int c = 0; c < nrhs; ++c) b[r * nrhs + c] -= fct * b[col * nrhs + c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    for (int c = 0; c < nrhs; ++c) {
      double s = b[r * nrhs + c];
      for (int q = r + 1; q < n; ++q) s -= a[r * n + q] * b[q * nrhs + c];
      b[r * nrhs + c] = s / a[r * n + r];
    }
  }
  return true;
}

}  // namespace

int compute_coeffs(int N, const double* sigma, double D, Coeffs* out, char* msg) {
  if (N < 2 || N > kMaxComp) {
    std::snprintf(msg, 256, "ncomp=%d outside 2..%d", N, kMaxComp);
    return -1;
  }
  if (!(D > 0.0)) {
    std::snprintf(msg, 256, "interface width D=%g must be positive", D);
    return -1;
  }
  Coeffs& c = *out;
  c = Coeffs();
  c.N = N;
  c.D = D;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const double s = sigma[i * N + j];
      if (i == j && s != 0.0) {
        std::snprintf(msg, 256, "sigma[%d][%d]=%g must be 0", i, i, s);
        return -1;
      }
      if (i != j && !(s > 0.0)) {
        std::snprintf(msg, 256, "sigma[%d][%d]=%g must be positive", i, j, s);
        return -1;
      }
      if (s != sigma[j * N + i]) {
        std::snprintf(msg, 256, "sigma is not symmetric at (%d,%d)", i, j);
        return -1;
      }
      c.sigma[i][j] = s;
      if (i != j) {
        c.beta[i][j] = 6.0 * s / D;
        c.kappa[i][j] = 3.0 * s * D / 4.0;
      }
    }

  // --- alpha, gamma from the bordered inverse
  {
    const int n = N + 1;
    std::vector<double> B(n * n, 0.0), X(n * n, 0.0);
    for (int i = 0; i < N; ++i) {
      for (int j = 0; j < N; ++j) B[i * n + j] = c.sigma[i][j];
      B[i * n + N] = 1.0;
      B[N * n + i] = 1.0;
    }
    for (int i = 0; i < n; ++i) X[i * n + i] = 1.0;
    if (!gauss_solve(B, n, X, n)) {
      std::snprintf(msg, 256, "bordered tension matrix is singular");
      return -2;
    }
    for (int i = 0; i < N; ++i) {
      for (int j = 0; j < N; ++j) c.alpha[i][j] = X[i * n + j];
      c.gamma[i] = -X[i * n + N];
    }
  }
  auto T = [&](int i, int j, int k, int l) {
    return c.alpha[i][j] * (c.sigma[j][k] + c.sigma[j][l]) +
           c.alpha[i][k] * (c.sigma[j][k] + c.sigma[k][l]) +
           c.alpha[i][l] * (c.sigma[j][l] + c.sigma[k][l]) - c.gamma[i];
  };

  // --- Lambda[j][triple] for every triple k<l<m (Eq. ngamma)
  auto& lam = c.lam;
  auto& th = c.theta;   // [k][l][j][m]
  for (int k = 0; k < N; ++k)
    for (int l = k + 1; l < N; ++l)
      for (int m = l + 1; m < N; ++m) {
        int S[kMaxComp], ns = 0;
        for (int j = 0; j < N; ++j)
          if (j != k && j != l && j != m) S[ns++] = j;
        if (ns == 0) continue;
        std::vector<double> A(ns * ns), rhs(ns);
        for (int r = 0; r < ns; ++r) {
          for (int q = 0; q < ns; ++q) A[r * ns + q] = c.alpha[S[r]][S[q]];
          rhs[r] = -6.0 * T(S[r], k, l, m);
        }
        if (!gauss_solve(A, ns, rhs, 1)) {
          std::snprintf(msg, 256, "alpha sub-matrix without {%d,%d,%d} is singular", k, l, m);
          return -2;
        }
        for (int r = 0; r < ns; ++r) lam[S[r]][k][l][m] = rhs[r];
      }

  // --- Theta[k][l][j][m], k<l, m outside {k,l}
  for (int k = 0; k < N; ++k)
    for (int l = k + 1; l < N; ++l)
      for (int m = 0; m < N; ++m) {
        if (m == k || m == l) continue;
        int S[kMaxComp], ns = 0;
        for (int j = 0; j < N; ++j)
          if (j != k && j != l && j != m) S[ns++] = j;
        if (ns == 0) continue;
        std::vector<double> A(ns * ns), rhs(ns);
        for (int r = 0; r < ns; ++r) {
          for (int q = 0; q < ns; ++q) A[r * ns + q] = c.alpha[S[r]][S[q]];
          rhs[r] = 2.0 * c.alpha[S[r]][m];
        }
        if (!gauss_solve(A, ns, rhs, 1)) {
          std::snprintf(msg, 256, "alpha sub-matrix without {%d,%d,%d} is singular", k, l, m);
          return -2;
        }
        for (int r = 0; r < ns; ++r) th[k][l][S[r]][m] = rhs[r];
      }

  auto sorted3 = [](int a, int b, int d, int* o) {
    int v[3] = {a, b, d};
    for (int x = 0; x < 3; ++x)
      for (int y = x + 1; y < 3; ++y)
        if (v[y] < v[x]) std::swap(v[x], v[y]);
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2];
  };

  for (int i = 0; i < N; ++i) {
    for (int l = 0; l < N; ++l)
      for (int m = l + 1; m < N; ++m) {
        if (l == i || m == i) continue;
        int t[3];
        sorted3(i, l, m, t);
        double acc = 6.0 * T(i, i, l, m);
        for (int j = 0; j < N; ++j)
          if (j != i && j != l && j != m) acc += c.alpha[i][j] * lam[j][t[0]][t[1]][t[2]];
        c.psi[i][l][m] = acc;
      }
    for (int k = 0; k < N; ++k)
      for (int l = k + 1; l < N; ++l) {
        if (k == i || l == i) continue;
        double acc = 2.0 * c.alpha[i][i];
        for (int j = 0; j < N; ++j)
          if (j != k && j != l && j != i) acc -= c.alpha[i][j] * th[k][l][j][i];
        c.xt[i][k][l] = acc;
      }
    for (int l = 0; l < N; ++l) {
      if (l == i) continue;
      const int a = i < l ? i : l, b = i < l ? l : i;
      for (int m = 0; m < N; ++m) {
        if (m == i || m == l) continue;
        double acc = 2.0 * c.alpha[i][m];
        for (int j = 0; j < N; ++j)
          if (j != i && j != l && j != m) acc -= c.alpha[i][j] * th[a][b][j][m];
        c.zt[i][l][m] = acc;
      }
    }
  }

  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j)
      for (int k = 0; k < N; ++k)
        if (k != i && k != j && c.sigma[i][j] - c.sigma[i][k] - c.sigma[j][k] > 0.0)
          c.any_positive_spreading = true;
  return 0;
}

}  // namespace nflbm
