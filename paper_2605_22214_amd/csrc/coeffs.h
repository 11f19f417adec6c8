// Host-side model coefficients of the N-component free-energy LBM.
// One-time FP64 precompute (Sec. II: "performed once for a given set of
// surface tensions").
#pragma once

namespace nflbm {

constexpr int kMaxComp = 8;

struct Coeffs {
  int N = 0;
  double D = 4.0;
  double sigma[kMaxComp][kMaxComp] = {};
  double beta[kMaxComp][kMaxComp] = {};   // 6 sigma / D (off-diagonal)
  double kappa[kMaxComp][kMaxComp] = {};  // 3 sigma D / 4 (off-diagonal)
  double alpha[kMaxComp][kMaxComp] = {};  // Eqs. alpha1, alpha2
  double gamma[kMaxComp] = {};
  // Factored flux-potential tables (entries outside the index sets are 0):
  //   psi[i][l][m] (l<m, l,m != i)   = 6 T_{i;ilm} + sum_{j not in ilm} alpha_ij Lambda_{j;ilm}
  //   xt[i][k][l]  (k<l, i not in kl) = 2 alpha_ii - sum_{j not in kli} alpha_ij Theta_{kl;j;i}
  //   zt[i][l][m]  (l != i, m not in il) = 2 alpha_im - sum_{j not in ilm} alpha_ij Theta_{il;j;m}
  double psi[kMaxComp][kMaxComp][kMaxComp] = {};
  double xt[kMaxComp][kMaxComp][kMaxComp] = {};
  double zt[kMaxComp][kMaxComp][kMaxComp] = {};
  // The solved coefficients themselves (user indices; 0 outside the index
  // sets): lam[j][k][l][m] = Lambda_{j;klm} for k<l<m without j (Eq. ngamma),
  // theta[k][l][j][m] = Theta_{kl;j;m} for k<l, j and m outside {k,l}, j != m.
  double lam[kMaxComp][kMaxComp][kMaxComp][kMaxComp] = {};
  double theta[kMaxComp][kMaxComp][kMaxComp][kMaxComp] = {};
  bool any_positive_spreading = false;    // some S_ij;k = s_ij - s_ik - s_jk > 0
};

// Returns 0 on success, -1 for an invalid sigma (not symmetric, non-zero
// diagonal, non-positive off-diagonal, N out of range, D <= 0), -2 if one of
// the linear systems is singular.  msg (>= 256 chars) receives the reason.
int compute_coeffs(int N, const double* sigma, double D, Coeffs* out, char* msg);

}  // namespace nflbm
