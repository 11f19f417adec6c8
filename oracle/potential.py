"""Free energy, chemical potentials and the flux potential mu~ (oracle, FP64).

Test infrastructure only.  All functions take concentrations C with shape
[N, ...] (any trailing lattice shape) and a ``Coefficients`` object.

Literal form (Sec. II):
  f(c) = c^2 (1-c)^2,  f'(c) = 2c(1 - 3c + 2c^2)                (Eq. FreeEnergy, Eq. mu)
  E_B  = sum_{i != j} (beta_ij / 2) [f(C_i) + f(C_j) - f(C_i + C_j)]
  mu_j = sum_{k != j} [beta_jk (f'(C_j) - f'(C_j + C_k)) + kappa_jk lap C_k]
  phi_j = (12/D) sum_{k<l<m, none equal j} Lambda_{j;jklm} C_k C_l C_m   (Eq. G)
  xi_j  = (12/D) Omega sum_{k<l, both != j} C_k^2 C_l^2
          (2 C_j - sum_{m != j,k,l} Theta_{kl;j;m} C_m)                    (Eq. P)
  mu~_i = sum_j alpha_ij (mu_j + phi_j + xi_j)                             (Eq. MU)

Factored form (the reading used by the time step, see step.py): the same
quantity regrouped with the tables of coeffs.py so that every non-gradient term
carries an explicit factor C_i:

  mu~_i = (3D/4) lap C_i
        + (12/D) C_i [ -(1 - 3 C_i + 2 C_i^2) + sum_{l<m; l,m != i} Psi_{i;lm} C_l C_m ]
        + (12/D) Omega C_i [ sum_{k<l; i not in {k,l}} X_{i;kl} C_k^2 C_l^2
                             + C_i sum_{l != i} C_l^2 sum_{m != i,l} Z_{i;l;m} C_m ]

The regrouping uses (a) sum_j alpha_ij kappa_jk = (3D/4)(delta_ik + gamma_i)
(from Eq. alpha1 with kappa = 3 sigma D / 4) and drops gamma_i lap(sum C),
which vanishes when sum_i C_i = 1; (b) Eq. fluxwrong, an identity on
sum_i C_i = 1; (c) Eq. ngamma, which removes every C_k C_l C_m term without
C_i; (d) the Theta system, which removes every xi term without C_i.  (d) needs
no sum rule.  With it an absent component (C_i = 0 on the stencil) has
mu~_i = 0 exactly in floating point, not only to rounding.
"""
import itertools

import numpy as np


def fpoly(c):
    return c * c * (1.0 - c) * (1.0 - c)


def fprime(c):
    return 2.0 * c * (1.0 - 3.0 * c + 2.0 * c * c)


def bulk_energy(C, co):
    """E_B of Eq. FreeEnergy, written as the double sum over ordered pairs."""
    N = co.N
    EB = np.zeros(C.shape[1:])
    for i in range(N):
        for j in range(N):
            if i == j:
                continue
            EB = EB + 0.5 * co.beta[i, j] * (fpoly(C[i]) + fpoly(C[j]) - fpoly(C[i] + C[j]))
    return EB


def mu_bulk(C, co):
    """Bulk part of mu_j: sum_{k != j} beta_jk (f'(C_j) - f'(C_j + C_k))."""
    N = co.N
    out = np.zeros_like(C)
    for j in range(N):
        for k in range(N):
            if k == j:
                continue
            out[j] = out[j] + co.beta[j, k] * (fprime(C[j]) - fprime(C[j] + C[k]))
    return out


def mu_full(C, lapC, co):
    """mu_j of Eq. mu, bulk plus gradient part."""
    N = co.N
    out = mu_bulk(C, co)
    for j in range(N):
        for k in range(N):
            if k == j:
                continue
            out[j] = out[j] + co.kappa[j, k] * lapC[k]
    return out


def phi(C, co):
    """phi_j of Eq. G."""
    N = co.N
    out = np.zeros_like(C)
    for j in range(N):
        for k, l, m in itertools.combinations(range(N), 3):
            if j in (k, l, m):
                continue
            out[j] = out[j] + co.Lam[j, k, l, m] * C[k] * C[l] * C[m]
    return (12.0 / co.D) * out


def xi(C, co, omega):
    """xi_j of Eq. P."""
    N = co.N
    out = np.zeros_like(C)
    if omega == 0.0:
        return out
    for j in range(N):
        for k, l in itertools.combinations(range(N), 2):
            if j in (k, l):
                continue
            inner = 2.0 * C[j]
            for m in range(N):
                if m in (j, k, l):
                    continue
                inner = inner - co.Theta[k, l, j, m] * C[m]
            out[j] = out[j] + C[k] ** 2 * C[l] ** 2 * inner
    return (12.0 / co.D) * omega * out


def mu_tilde_literal(C, lapC, co, omega=0.0, with_phi=True, with_xi=True):
    """mu~_i = sum_j alpha_ij (mu_j + phi_j + xi_j), Eq. MU written out."""
    N = co.N
    s = mu_full(C, lapC, co)
    if with_phi:
        s = s + phi(C, co)
    if with_xi:
        s = s + xi(C, co, omega)
    out = np.zeros_like(C)
    for i in range(N):
        for j in range(N):
            out[i] = out[i] + co.alpha[i, j] * s[j]
    return out


def flux_potentials(C, lapC, co, omega=0.0):
    """mu_j + phi_j + xi_j for every component j: the quantity that Eq. MU
    contracts with alpha, and whose gradient the concentration-dependent
    mobility of Appendix C contracts with the per-node alpha."""
    return mu_full(C, lapC, co) + phi(C, co) + xi(C, co, omega)


def alpha_c2c2(C):
    """Concentration-dependent mobility matrix of Appendix C at every node:
    alpha_ij = C_i^2 C_j^2 for i != j and alpha_ii = -sum_{j != i} alpha_ij,
    so that every row (and column) sums to zero -> [N, N, ...]."""
    N = C.shape[0]
    a = np.zeros((N, N) + C.shape[1:])
    for i in range(N):
        for j in range(N):
            if j != i:
                a[i, j] = C[i] ** 2 * C[j] ** 2
                a[i, i] = a[i, i] - a[i, j]
    return a


def bulk_flux_potential_eq_fluxwrong(C, co):
    """The right-hand side of Eq. fluxwrong without the gradient:
    (12/D) [ -C_i (1 - 3C_i + 2C_i^2) + 6 sum_{j<k<l} T_{i;jkl} C_j C_k C_l ].
    Holds for sum_j alpha_ij mu_{j,b} on sum_i C_i = 1."""
    N = co.N
    out = np.zeros_like(C)
    for i in range(N):
        acc = -C[i] * (1.0 - 3.0 * C[i] + 2.0 * C[i] ** 2)
        for j, k, l in itertools.combinations(range(N), 3):
            acc = acc + 6.0 * co.T[i, j, k, l] * C[j] * C[k] * C[l]
        out[i] = acc
    return (12.0 / co.D) * out


def mu_tilde_factored(C, lapC, co, omega=0.0):
    """mu~_i in the factored form (module docstring)."""
    N = co.N
    out = np.zeros_like(C)
    for i in range(N):
        bracket = -(1.0 - 3.0 * C[i] + 2.0 * C[i] * C[i])
        for l, m in itertools.combinations([q for q in range(N) if q != i], 2):
            bracket = bracket + co.Psi[i, l, m] * C[l] * C[m]
        val = (3.0 * co.D / 4.0) * lapC[i] + (12.0 / co.D) * C[i] * bracket
        if omega != 0.0:
            sx = np.zeros_like(C[i])
            for k, l in itertools.combinations([q for q in range(N) if q != i], 2):
                sx = sx + co.X[i, k, l] * C[k] ** 2 * C[l] ** 2
            sy = np.zeros_like(C[i])
            for l in range(N):
                if l == i:
                    continue
                inner = np.zeros_like(C[i])
                for m in range(N):
                    if m in (i, l):
                        continue
                    inner = inner + co.Z[i, l, m] * C[m]
                sy = sy + C[l] ** 2 * inner
            val = val + (12.0 / co.D) * omega * C[i] * (sx + C[i] * sy)
        out[i] = val
    return out
