"""Model coefficients of the oracle (FP64, NumPy).  Test infrastructure only.

Everything here is a one-time host computation from the pairwise surface
tensions sigma_ij and the interface width D (Sec. II):

* beta_ij, kappa_ij: inverted from D = sqrt(8 kappa/beta) and
  sigma = sqrt(2 kappa beta / 9) (text after Eq. FreeEnergy):
  beta = 6 sigma / D, kappa = 3 sigma D / 4.
* alpha, gamma: the linear system of Eqs. alpha1 and alpha2,
  alpha sigma = I + gamma 1^T and alpha 1 = 0, solved as one (N^2+N) system.
* T_{i;jkl}: the coefficient of C_j C_k C_l in Eq. fluxwrong.
* Lambda_{j;jklm}: for every triple {k,l,m}, the system of Eq. ngamma,
  sum_{j not in klm} alpha_ij Lambda_j = Gamma_{i,klm} for i not in {k,l,m},
  with Gamma_{i,klm} = -6 T_{i;klm}.
* Theta_{kl;j;m}: for every pair {k,l} and m outside it, the system printed
  after Eq. P, sum_{j not in klm} alpha_ij Theta_{kl;j;m} = 2 alpha_im.
* S_{ij;k}: the spreading parameters of Eq. spreading.

The factored tables Psi, X and Z regroup sum_j alpha_ij (mu_j + phi_j + xi_j)
so that mu~_i is an explicit multiple of C_i (see potential.py):

  Psi_{i;lm} = 6 T_{i;ilm} + sum_{j not in {i,l,m}} alpha_ij Lambda_{j;{ilm}}
  X_{i;kl}   = 2 alpha_ii - sum_{j not in {k,l,i}} alpha_ij Theta_{kl;j;i}
  Z_{i;l;m}  = 2 alpha_im - sum_{j not in {i,l,m}} alpha_ij Theta_{{il};j;m}

Undefined entries of the dense arrays are NaN so that any use of one shows.
"""
import itertools

import numpy as np


class Coefficients:
    """All tables for one (sigma, D).  Arrays are dense and indexed from 0."""

    def __init__(self, sigma, D=4.0):
        sigma = np.array(sigma, dtype=np.float64)
        N = sigma.shape[0]
        if sigma.shape != (N, N) or N < 2:
            raise ValueError("sigma must be a square N x N matrix with N >= 2")
        if not np.allclose(sigma, sigma.T, rtol=0, atol=0):
            raise ValueError("sigma must be symmetric")
        if np.any(np.diag(sigma) != 0.0):
            raise ValueError("sigma must have a zero diagonal")
        off = sigma[~np.eye(N, dtype=bool)]
        if np.any(off <= 0.0):
            raise ValueError("off-diagonal sigma must be positive")
        self.N = N
        self.D = float(D)
        self.sigma = sigma
        self.beta = 6.0 * sigma / self.D
        self.kappa = 3.0 * sigma * self.D / 4.0
        self.alpha, self.gamma = solve_alpha_gamma(sigma)
        self.T = triple_T(self.alpha, self.gamma, sigma)
        self.Lam = solve_lambda(self.alpha, self.T)
        self.Theta = solve_theta(self.alpha)
        self.Psi, self.X, self.Z = factored_tables(self.alpha, self.T, self.Lam, self.Theta)
        self.spreading = spreading_parameters(sigma)


def solve_alpha_gamma(sigma):
    """Eqs. alpha1 and alpha2 as one linear system in (alpha, gamma).

    Unknown vector: alpha in row-major order (N*N entries), then gamma (N).
    Rows 0..N*N-1: sum_j alpha_ij sigma_jk - gamma_i = delta_ik.
    Rows N*N..N*N+N-1: sum_j alpha_ij = 0.
    """
    N = sigma.shape[0]
    n = N * N + N
    A = np.zeros((n, n))
    b = np.zeros(n)
    for i in range(N):
        for k in range(N):
            r = i * N + k
            for j in range(N):
                A[r, i * N + j] = sigma[j, k]
            A[r, N * N + i] = -1.0
            b[r] = 1.0 if i == k else 0.0
    for i in range(N):
        r = N * N + i
        for j in range(N):
            A[r, i * N + j] = 1.0
    x = np.linalg.solve(A, b)
    return x[: N * N].reshape(N, N), x[N * N:].copy()


def triple_T(alpha, gamma, sigma):
    """T[i, j, k, l] for distinct j, k, l (any order; T is symmetric in them).

    The bracket of Eq. fluxwrong:
    alpha_ij (s_jk + s_jl) + alpha_ik (s_jk + s_kl) + alpha_il (s_jl + s_kl) - gamma_i.
    """
    N = alpha.shape[0]
    T = np.full((N, N, N, N), np.nan)
    for i in range(N):
        for j, k, l in itertools.permutations(range(N), 3):
            T[i, j, k, l] = (alpha[i, j] * (sigma[j, k] + sigma[j, l])
                             + alpha[i, k] * (sigma[j, k] + sigma[k, l])
                             + alpha[i, l] * (sigma[j, l] + sigma[k, l])
                             - gamma[i])
    return T


def solve_lambda(alpha, T):
    """Lam[j, k, l, m] (k<l<m, j outside) from Eq. ngamma for every triple."""
    N = alpha.shape[0]
    Lam = np.full((N, N, N, N), np.nan)
    for k, l, m in itertools.combinations(range(N), 3):
        S = [j for j in range(N) if j not in (k, l, m)]
        if not S:
            continue
        Gamma = np.array([-6.0 * T[i, k, l, m] for i in S])
        sub = alpha[np.ix_(S, S)]
        lam = np.linalg.solve(sub, Gamma)
        for idx, j in enumerate(S):
            Lam[j, k, l, m] = lam[idx]
    return Lam


def solve_theta(alpha):
    """Theta[k, l, j, m] (k<l; j, m distinct and outside {k,l}).

    For each pair {k,l} and each m outside it:
    sum_{j not in {k,l,m}} alpha_ij Theta_{kl;j;m} = 2 alpha_im, i not in {k,l,m}.
    """
    N = alpha.shape[0]
    Th = np.full((N, N, N, N), np.nan)
    for k, l in itertools.combinations(range(N), 2):
        for m in range(N):
            if m in (k, l):
                continue
            S = [j for j in range(N) if j not in (k, l, m)]
            if not S:
                continue
            sub = alpha[np.ix_(S, S)]
            rhs = 2.0 * alpha[S, m]
            th = np.linalg.solve(sub, rhs)
            for idx, j in enumerate(S):
                Th[k, l, j, m] = th[idx]
    return Th


def factored_tables(alpha, T, Lam, Theta):
    """Psi[i,l,m] (l<m, both != i), X[i,k,l] (k<l, i outside), Z[i,l,m]."""
    N = alpha.shape[0]
    Psi = np.full((N, N, N), np.nan)
    X = np.full((N, N, N), np.nan)
    Z = np.full((N, N, N), np.nan)
    for i in range(N):
        for l, m in itertools.combinations([q for q in range(N) if q != i], 2):
            trip = tuple(sorted((i, l, m)))
            acc = 6.0 * T[i, i, l, m]
            for j in range(N):
                if j in trip:
                    continue
                acc += alpha[i, j] * Lam[j, trip[0], trip[1], trip[2]]
            Psi[i, l, m] = acc
        for k, l in itertools.combinations([q for q in range(N) if q != i], 2):
            acc = 2.0 * alpha[i, i]
            for j in range(N):
                if j in (k, l, i):
                    continue
                acc -= alpha[i, j] * Theta[k, l, j, i]
            X[i, k, l] = acc
        for l in range(N):
            if l == i:
                continue
            a, b = min(i, l), max(i, l)
            for m in range(N):
                if m in (i, l):
                    continue
                acc = 2.0 * alpha[i, m]
                for j in range(N):
                    if j in (i, l, m):
                        continue
                    acc -= alpha[i, j] * Theta[a, b, j, m]
                Z[i, l, m] = acc
    return Psi, X, Z


def spreading_parameters(sigma):
    """S[(i,j,k)] = sigma_ij - sigma_ik - sigma_jk for i<j, k outside (Eq. spreading)."""
    N = sigma.shape[0]
    out = {}
    for i, j in itertools.combinations(range(N), 2):
        for k in range(N):
            if k in (i, j):
                continue
            out[(i, j, k)] = sigma[i, j] - sigma[i, k] - sigma[j, k]
    return out


def equal_sigma(N, s):
    """Matrix with every off-diagonal tension equal to s."""
    return s * (np.ones((N, N)) - np.eye(N))
