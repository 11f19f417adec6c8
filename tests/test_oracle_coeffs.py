"""Pins of the oracle's coefficient tables against closed forms (CPU only).

Each expected value below is derived by hand from the defining equations, not
by re-running the oracle's routine:

* N = 2: alpha = (1/(2 s)) [[-1, 1], [1, -1]], gamma = -1/2 (Eqs. alpha1/alpha2).
* Equal tensions sigma = s (J - I): alpha = -(I - J/N)/s and gamma = -1/N
  (check: -(I - J/N)(J - I) = I - J/N).
* Equal tensions, Eq. ngamma: T_{i;klm} = 7/N for i outside the triple, so
  Gamma = -42/N, and alpha[S,S] (const) = -(3/N)/s * const gives Lambda = 14 s.
* Equal tensions, the Theta system: 2 alpha_im = 2/(N s) gives Theta = -2/3.
* beta, kappa invert D = sqrt(8 kappa/beta) and sigma = sqrt(2 kappa beta / 9).
"""
import numpy as np
import pytest

from oracle.coeffs import Coefficients, equal_sigma


def random_sigma(N, rng, lo=0.003, hi=0.009):
    s = rng.uniform(lo, hi, size=(N, N))
    s = 0.5 * (s + s.T)
    np.fill_diagonal(s, 0.0)
    return s


def test_binary_closed_form():
    s = 0.0073
    co = Coefficients(equal_sigma(2, s))
    expect = np.array([[-1.0, 1.0], [1.0, -1.0]]) / (2 * s)
    np.testing.assert_allclose(co.alpha, expect, rtol=1e-13)
    np.testing.assert_allclose(co.gamma, [-0.5, -0.5], rtol=1e-13)


@pytest.mark.parametrize("N", [3, 4, 5, 6, 7, 8])
def test_equal_sigma_closed_forms(N):
    s = 0.004
    co = Coefficients(equal_sigma(N, s))
    I, J = np.eye(N), np.ones((N, N))
    np.testing.assert_allclose(co.alpha, -(I - J / N) / s, rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(co.gamma, -np.ones(N) / N, rtol=1e-12)
    lam = co.Lam[~np.isnan(co.Lam)]
    th = co.Theta[~np.isnan(co.Theta)]
    if N >= 4:
        assert lam.size > 0 and th.size > 0
        np.testing.assert_allclose(lam, 14 * s, rtol=1e-11)
        np.testing.assert_allclose(th, -2.0 / 3.0, rtol=1e-11)
    else:
        assert lam.size == 0 and th.size == 0


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 7, 8])
def test_alpha_identities_random(N):
    rng = np.random.default_rng(100 + N)
    sig = random_sigma(N, rng)
    co = Coefficients(sig)
    a, g = co.alpha, co.gamma
    scale = np.abs(a).max()
    # Eq. alpha1 and Eq. alpha2
    np.testing.assert_allclose(a @ sig, np.eye(N) + np.outer(g, np.ones(N)), atol=1e-12)
    np.testing.assert_allclose(a @ np.ones(N), 0.0, atol=1e-12 * scale)
    # symmetric, negative semidefinite with the single null vector 1
    np.testing.assert_allclose(a, a.T, atol=1e-12 * scale)
    ev = np.linalg.eigvalsh(a)
    assert np.sum(np.abs(ev) < 1e-9 * scale) == 1
    assert np.all(ev < 1e-9 * scale)


@pytest.mark.parametrize("N", [4, 5, 6])
def test_lambda_theta_solve_their_systems(N):
    """Residuals of Eq. ngamma and of the Theta system, built row by row from
    the printed equations (not from the oracle's solve)."""
    rng = np.random.default_rng(7 + N)
    sig = random_sigma(N, rng)
    co = Coefficients(sig)
    a, g = co.alpha, co.gamma
    import itertools
    for k, l, m in itertools.combinations(range(N), 3):
        S = [j for j in range(N) if j not in (k, l, m)]
        for i in S:
            Gam = -6 * (a[i, k] * (sig[k, l] + sig[k, m]) + a[i, l] * (sig[k, l] + sig[l, m])
                        + a[i, m] * (sig[k, m] + sig[l, m]) - g[i])
            lhs = sum(a[i, j] * co.Lam[j, k, l, m] for j in S)
            assert abs(lhs - Gam) < 1e-10 * max(1.0, abs(Gam))
    for k, l in itertools.combinations(range(N), 2):
        for m in range(N):
            if m in (k, l):
                continue
            S = [j for j in range(N) if j not in (k, l, m)]
            for i in S:
                lhs = sum(a[i, j] * co.Theta[k, l, j, m] for j in S)
                assert abs(lhs - 2 * a[i, m]) < 1e-10 * max(1.0, abs(a[i, m]))


def test_beta_kappa_inversion():
    rng = np.random.default_rng(3)
    sig = random_sigma(4, rng)
    for D in (3.0, 4.0, 5.5):
        co = Coefficients(sig, D)
        off = ~np.eye(4, dtype=bool)
        np.testing.assert_allclose(np.sqrt(8 * co.kappa[off] / co.beta[off]), D, rtol=1e-14)
        np.testing.assert_allclose(np.sqrt(2 * co.kappa[off] * co.beta[off] / 9), sig[off],
                                   rtol=1e-14)


@pytest.mark.parametrize("N", [3, 4, 6])
def test_alpha_kappa_identity(N):
    """sum_j alpha_ij kappa_jk = (3D/4)(delta_ik + gamma_i): the gradient part of
    mu~ is (3D/4)(lap C_i + gamma_i lap sum C)."""
    rng = np.random.default_rng(11 + N)
    co = Coefficients(random_sigma(N, rng))
    lhs = co.alpha @ co.kappa
    rhs = 0.75 * co.D * (np.eye(N) + np.outer(co.gamma, np.ones(N)))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_spreading_parameters():
    sig = equal_sigma(3, 0.005)
    sig[0, 2] = sig[2, 0] = 0.012
    co = Coefficients(sig)
    assert co.spreading[(0, 2, 1)] == pytest.approx(0.012 - 0.005 - 0.005)
    assert co.spreading[(0, 1, 2)] == pytest.approx(0.005 - 0.012 - 0.005)


def test_rejects_bad_sigma():
    with pytest.raises(ValueError):
        Coefficients(np.array([[0, 0.01], [0.02, 0]]))
    with pytest.raises(ValueError):
        Coefficients(np.array([[0.1, 0.01], [0.01, 0]]))
    with pytest.raises(ValueError):
        Coefficients(np.array([[0, -0.01], [-0.01, 0]]))
