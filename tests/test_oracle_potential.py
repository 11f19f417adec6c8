"""Pins of the oracle's free energy and flux potential (CPU only).

* Eq. fluxwrong is printed as an identity for sum_j alpha_ij mu_{j,b} on the
  simplex; the oracle's literal mu_b must satisfy it.
* The factored mu~ (explicit factor C_i) must equal Eq. MU written out
  (sum_j alpha_ij (mu_j + phi_j + xi_j)) wherever sum_i C_i = 1.
* Fig. 1 (Sec. II): without phi an absent fourth component sees a non-zero
  bulk potential where three others meet; with phi it is zero.  In the
  factored form it is exactly 0.0.
* Reduction (Sec. I, Sec. II): an N-system with C_N = 0 reproduces the
  (N-1)-system built from the sigma sub-matrix.
* The free energy of a flat binary interface C = 1/2 [1 + tanh(2z/D)]
  integrates to sigma_12 (text after Eq. FreeEnergy); this pins beta, kappa,
  the pair sum of E_B and the sign of E_I.
"""
import itertools

import numpy as np
import pytest

from oracle import potential as pot
from oracle.coeffs import Coefficients, equal_sigma


def random_sigma(N, rng, lo=0.003, hi=0.009):
    s = rng.uniform(lo, hi, size=(N, N))
    s = 0.5 * (s + s.T)
    np.fill_diagonal(s, 0.0)
    return s


def simplex(N, n, rng):
    C = rng.uniform(0.0, 1.0, size=(N, n))
    return C / C.sum(axis=0)


@pytest.mark.parametrize("N", [3, 4, 5, 6, 7])
def test_eq_fluxwrong_identity(N):
    rng = np.random.default_rng(N)
    co = Coefficients(random_sigma(N, rng))
    C = simplex(N, 300, rng)
    lhs = co.alpha @ pot.mu_bulk(C, co)
    rhs = pot.bulk_flux_potential_eq_fluxwrong(C, co)
    assert np.abs(lhs - rhs).max() < 1e-12 * max(1.0, np.abs(rhs).max())


def test_eq_fluxwrong_written_out_for_n3():
    """For N = 3 the single triple of Eq. fluxwrong is Eq. fluxright."""
    rng = np.random.default_rng(5)
    sig = random_sigma(3, rng)
    co = Coefficients(sig)
    C = simplex(3, 50, rng)
    a, g = co.alpha, co.gamma
    for i in range(3):
        j, k = [q for q in range(3) if q != i]
        coef = 6 * (a[i, i] * (sig[i, j] + sig[i, k]) + a[i, j] * (sig[i, j] + sig[j, k])
                    + a[i, k] * (sig[i, k] + sig[j, k]) - g[i])
        expect = 12 / co.D * (-C[i] * (1 - 3 * C[i] + 2 * C[i] ** 2) + coef * C[0] * C[1] * C[2])
        got = (co.alpha @ pot.mu_bulk(C, co))[i]
        np.testing.assert_allclose(got, expect, atol=1e-12)


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 8])
@pytest.mark.parametrize("omega", [0.0, 1.0 / 18.0])
def test_factored_equals_literal_on_simplex(N, omega):
    rng = np.random.default_rng(20 + N)
    co = Coefficients(random_sigma(N, rng))
    C = simplex(N, 400, rng)
    lap = rng.normal(size=(N, 400))
    lap -= lap.mean(axis=0)           # lap of sum C vanishes when sum C = 1
    lit = pot.mu_tilde_literal(C, lap, co, omega)
    fac = pot.mu_tilde_factored(C, lap, co, omega)
    assert np.abs(lit - fac).max() < 1e-12 * np.abs(lit).max()


@pytest.mark.parametrize("N", [4, 5, 6])
def test_absent_component_potential(N):
    rng = np.random.default_rng(40 + N)
    co = Coefficients(random_sigma(N, rng))
    C = simplex(N - 1, 500, rng)
    C = np.concatenate([C, np.zeros((1, 500))])
    lap = rng.normal(size=(N, 500))
    lap[-1] = 0.0
    lap[:-1] -= lap[:-1].mean(axis=0)
    fac = pot.mu_tilde_factored(C, lap, co, 1.0 / 18.0)
    assert np.all(fac[-1] == 0.0)                           # exact, not to rounding
    lit = pot.mu_tilde_literal(C, lap, co, 1.0 / 18.0)
    assert np.abs(lit[-1]).max() < 1e-12 * np.abs(lit).max()
    nophi = pot.mu_tilde_literal(C, np.zeros_like(lap), co, 0.0, with_phi=False)
    assert np.abs(nophi[-1]).max() > 1e-2                   # Fig. 1(a): nucleation drive


def test_absent_potential_without_phi_vanishes_for_three_components():
    """For N = 3 alpha alone is reduction consistent (text after Eq. fluxright)."""
    rng = np.random.default_rng(9)
    co = Coefficients(random_sigma(3, rng))
    C = simplex(2, 100, rng)
    C = np.concatenate([C, np.zeros((1, 100))])
    nophi = pot.mu_tilde_literal(C, np.zeros_like(C), co, 0.0, with_phi=False)
    assert np.abs(nophi[-1]).max() < 1e-13


@pytest.mark.parametrize("N", [4, 5, 6])
def test_reduction_to_smaller_system(N):
    rng = np.random.default_rng(60 + N)
    sig = random_sigma(N, rng)
    big = Coefficients(sig)
    small = Coefficients(sig[:-1, :-1])
    Cs = simplex(N - 1, 300, rng)
    lap = rng.normal(size=(N - 1, 300))
    lap -= lap.mean(axis=0)
    Cb = np.concatenate([Cs, np.zeros((1, 300))])
    lapb = np.concatenate([lap, np.zeros((1, 300))])
    for omega in (0.0, 1.0 / 18.0):
        mb = pot.mu_tilde_factored(Cb, lapb, big, omega)
        ms = pot.mu_tilde_factored(Cs, lap, small, omega)
        assert np.abs(mb[:-1] - ms).max() < 1e-12 * np.abs(ms).max()


@pytest.mark.parametrize("N", [2, 3])
def test_flat_interface_energy_is_sigma(N):
    D, s12 = 4.0, 0.0067
    sig = equal_sigma(N, 0.005)
    sig[0, 1] = sig[1, 0] = s12
    co = Coefficients(sig, D)
    h = 1e-3
    z = np.arange(-40.0, 40.0, h)
    c1 = 0.5 * (1 + np.tanh(2 * z / D))
    C = np.zeros((N, z.size))
    C[0], C[1] = c1, 1 - c1
    EB = pot.bulk_energy(C, co)
    grad = np.gradient(C, h, axis=1)
    EI = np.zeros_like(z)
    for i, j in itertools.permutations(range(N), 2):
        EI -= 0.5 * co.kappa[i, j] * grad[i] * grad[j]
    excess = np.trapezoid(EB + EI, z)
    assert excess == pytest.approx(s12, rel=1e-6)


def test_fprime_is_derivative_of_f():
    c = np.linspace(-0.5, 1.5, 101)
    h = 1e-6
    num = (pot.fpoly(c + h) - pot.fpoly(c - h)) / (2 * h)
    np.testing.assert_allclose(pot.fprime(c), num, atol=1e-8)


def test_mu_bulk_is_derivative_of_eb():
    rng = np.random.default_rng(1)
    co = Coefficients(random_sigma(4, rng))
    C = rng.uniform(-0.1, 1.1, size=(4, 20))
    mb = pot.mu_bulk(C, co)
    h = 1e-6
    for j in range(4):
        dp, dm = C.copy(), C.copy()
        dp[j] += h
        dm[j] -= h
        num = (pot.bulk_energy(dp, co) - pot.bulk_energy(dm, co)) / (2 * h)
        np.testing.assert_allclose(mb[j], num, atol=1e-9)
