"""Pins of the oracle's concentration-dependent mobility variant (Appendix C)
on the CPU.

  alpha(C)             alpha_ij = C_i^2 C_j^2, alpha_ii = -sum_{j != i}: symmetric,
                       rows summing to zero, negative semidefinite, the N = 2
                       closed form, an absent component's row exactly zero
  linear dispersion    a Fourier mode about a uniform, unequal mixture grows by
                       the closed-form matrix of analysis.source_mobility_growth
                       (source factor, its sign, alpha's indices and the gradient
                       of mu + phi + xi all enter it)
  conservation         per-component mass and sum_i C_i = 1, also with walls and
                       tau_g != 1
  reduction            an absent component stays exactly 0.0, and an N-system
                       with an absent component follows the (N-1)-system
"""
import numpy as np
import pytest

import workloads as W
from oracle import analysis as A
from oracle import potential as pot
from oracle import step as S
from oracle.coeffs import Coefficients
from oracle.lattice import D2Q9, D3Q19


def random_sigma(N, seed, lo=0.004, hi=0.008):
    rng = np.random.default_rng(seed)
    s = rng.uniform(lo, hi, size=(N, N))
    s = 0.5 * (s + s.T)
    np.fill_diagonal(s, 0.0)
    return s


def test_alpha_c2c2_properties():
    rng = np.random.default_rng(1)
    for N in (2, 3, 5, 6):
        C = rng.uniform(0.0, 1.0, size=(N, 7))
        C /= C.sum(axis=0, keepdims=True)
        a = pot.alpha_c2c2(C)
        for p in range(C.shape[1]):
            ap = a[:, :, p]
            assert np.array_equal(ap, ap.T)
            assert np.abs(ap.sum(axis=1)).max() <= 1e-16
            ev = np.linalg.eigvalsh(ap)
            assert ev.max() <= 1e-17
            for i in range(N):
                for j in range(N):
                    if i != j:
                        assert ap[i, j] == C[i, p] ** 2 * C[j, p] ** 2
    C = np.array([[0.3], [0.7]])
    q = 0.3 ** 2 * 0.7 ** 2
    assert np.allclose(pot.alpha_c2c2(C)[:, :, 0], q * np.array([[-1.0, 1.0], [1.0, -1.0]]),
                       rtol=1e-15, atol=0)
    C = np.array([[0.5], [0.0], [0.5]])
    a = pot.alpha_c2c2(C)[:, :, 0]
    assert np.all(a[1] == 0.0) and np.all(a[:, 1] == 0.0)


@pytest.mark.parametrize("N,omega", [(3, 0.0), (4, 1.0 / 18.0), (6, 1.0 / 90.0)])
def test_flux_potentials_contract_to_factored_mu(N, omega):
    """sum_j alpha_ij (mu_j + phi_j + xi_j) with the constant alpha equals the
    factored mu~_i, which is written from different tables (on sum C = 1 and
    a Laplacian field that sums to zero over components)."""
    rng = np.random.default_rng(30 + N)
    co = Coefficients(random_sigma(N, 40 + N))
    C = rng.uniform(0.0, 1.0, size=(N, 50))
    C /= C.sum(axis=0, keepdims=True)
    lap = rng.standard_normal((N, 50)) * 1e-2
    lap -= lap.mean(axis=0, keepdims=True)
    Phi = pot.flux_potentials(C, lap, co, omega)
    lhs = np.einsum("ij,jp->ip", co.alpha, Phi)
    rhs = pot.mu_tilde_factored(C, lap, co, omega)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


def bulk_jacobian(C0, co, omega=0.0, h=1e-5):
    """d(mu_j + phi_j + xi_j)/dC_l at a uniform C0 with lap C = 0 (central
    differences; every C_l an independent variable)."""
    N = len(C0)
    J = np.zeros((N, N))
    z = np.zeros((N, 1))
    for l in range(N):
        dp = np.array(C0, dtype=np.float64).reshape(N, 1)
        dm = dp.copy()
        dp[l] += h
        dm[l] -= h
        J[:, l] = (pot.flux_potentials(dp, z, co, omega)[:, 0]
                   - pot.flux_potentials(dm, z, co, omega)[:, 0]) / (2 * h)
    return J


@pytest.mark.parametrize("lat,shape,kidx,omega", [
    (D2Q9, (32, 32, 1), (4, 3, 0), 0.0),
    (D2Q9, (24, 16, 1), (5, -2, 0), 1.0 / 18.0),
    (D3Q19, (16, 12, 10), (3, 2, 1), 0.0),
])
def test_c2c2_linear_dispersion(lat, shape, kidx, omega):
    """One cosine mode of amplitude 1e-7 about C0 = (0.4, 0.3, 0.2, 0.1) with
    unequal tensions, 300 steps without hydrodynamics: the mode's amplitude
    vector against M(k)^t applied to the initial one."""
    N, T = 4, 300
    nx, ny, nz = shape
    sigma = random_sigma(N, 21)
    co = Coefficients(sigma)
    C0 = np.array([0.4, 0.3, 0.2, 0.1])
    u = np.array([1.0, -2.0, 0.5, 0.5])
    kvec = [2 * np.pi * kidx[0] / nx, 2 * np.pi * kidx[1] / ny, 2 * np.pi * kidx[2] / nz]
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phase = kvec[0] * x + kvec[1] * y + kvec[2] * z
    eps = 1e-7
    C = C0[:, None, None, None] + eps * u[:, None, None, None] * np.cos(phase)[None]
    par = S.Params(lat, shape, sigma, np.ones(N), m=0.1, hydro=False, mobility="c2c2",
                   m_star=10.0, omega_stab=omega)
    f, g = S.initial_state(par, C)
    for _ in range(T):
        f, g, _ = S.step(f, g, par)
    Ct = S.concentrations(g, par)
    nodes = nx * ny * nz
    amp_c = 2.0 * (Ct - C0[:, None, None, None]).reshape(N, -1) @ np.cos(phase).ravel() / nodes
    amp_s = 2.0 * (Ct - C0[:, None, None, None]).reshape(N, -1) @ np.sin(phase).ravel() / nodes
    alpha0 = pot.alpha_c2c2(C0.reshape(N, 1))[:, :, 0]
    M = A.source_mobility_growth(lat, kvec, alpha0, bulk_jacobian(C0, co, omega), co.kappa, 10.0)
    pred = np.linalg.matrix_power(M, T) @ (eps * u)
    change = pred - eps * u
    assert np.abs(change).max() > 1e-3 * eps          # the mode really evolves
    assert np.abs(amp_c - pred).max() <= 1e-4 * np.abs(change).max()
    assert np.abs(amp_s).max() <= 1e-6 * eps


def c2c2_params(w, **kw):
    return S.Params(D2Q9 if w["lattice"] == "D2Q9" else D3Q19, w["shape"], w["sigma"], w["tau"],
                    tau_g=w.get("tau_g"), m=w["m"], walls=w["walls"], mobility="c2c2",
                    m_star=10.0, **kw)


@pytest.mark.parametrize("hydro,walls,tau_g", [(False, (False, False, False), 1.0),
                                               (True, (False, True, False), 1.0),
                                               (True, (False, False, False), 0.8)])
def test_c2c2_conservation(hydro, walls, tau_g):
    w = W.coarsening_2d(20, 3, seed=4)
    w["walls"] = walls
    w["tau_g"] = np.full(3, tau_g)
    par = c2c2_params(w, hydro=hydro)
    f, g = S.initial_state(par, w["C0"])
    C0 = S.concentrations(g, par)
    for _ in range(60):
        f, g, mac = S.step(f, g, par)
    C = S.concentrations(g, par)
    mass0, mass = C0.sum(axis=(1, 2, 3)), C.sum(axis=(1, 2, 3))
    assert np.abs(mass - mass0).max() <= 1e-13 * mass0.max()
    assert np.abs(C.sum(axis=0) - 1.0).max() <= 1e-14
    assert np.abs(mac["G"].sum(axis=0)).max() <= 1e-15 * max(np.abs(mac["G"]).max(), 1e-300) * 10
    assert np.abs(C - C0).max() > 1e-4                 # the variant moves C


def test_c2c2_absent_component_and_reduction():
    """N = 4 with C_4 = 0 against the N = 3 system with the sigma sub-matrix,
    both with the concentration-dependent mobility, hydrodynamics on."""
    s = random_sigma(4, 8)
    w3 = W.lens_2d(20, 16, radius=4.0, sigma=s[:3, :3])
    w4 = dict(w3)
    w4["sigma"] = s
    w4["C0"] = np.concatenate([w3["C0"], np.zeros((1,) + w3["C0"].shape[1:])])
    w4["tau"] = np.ones(4)
    w4["tau_g"] = np.ones(4)
    p3 = c2c2_params(w3, implicit=0)
    p4 = c2c2_params(w4, implicit=0)
    f3, g3 = S.initial_state(p3, w3["C0"])
    f4, g4 = S.initial_state(p4, w4["C0"])
    for _ in range(100):
        f3, g3, _ = S.step(f3, g3, p3)
        f4, g4, _ = S.step(f4, g4, p4)
    assert np.all(g4[3] == 0.0)
    assert np.abs(g4[:3] - g3).max() < 1e-12 * np.abs(g3).max()
    assert np.abs(f4[1:] - f3[1:]).max() < 1e-10 * np.abs(f3).max()
