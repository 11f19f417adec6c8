"""Pins of the oracle's open faces (Sec. III C: velocity Dirichlet for f,
anti-bounce-back concentration Dirichlet for g) on the CPU.

  Couette        a wall at y = -1/2 and an open face at y = ny - 1/2 moving
                 with U: the steady profile of halfway bounce-back with the
                 moving-wall correction is exactly u_x = U (y + 1/2) / ny
                 (a wrong sign of the correction gives -U)
  plug flow      open faces on x- and x+ with v_b = u and C_b = the interior
                 mixture: the uniform state (C_b, v = u) is an exact fixed
                 point, which holds only with the even part of g^eq in the
                 anti-bounce-back rule and the f correction's sign
  mass balance   through an open face a component's mass changes only by what
                 crosses it: with v_b = 0 on both faces of a closed channel and
                 C_b equal to the initial interior values, nothing enters
  outflow        the convective outflow (Eq. convect) lets a pulse carried by
                 the flow leave with far less reflection than a velocity-
                 Dirichlet outlet, and inlet + outflow keep a uniform plug
                 flow exactly; mirrored in x (inlet on x+, outflow on x-) a
                 three-component run gives the mirrored fields, which pins
                 the outward normal and the planes of the x- face
"""
import numpy as np
import pytest

import workloads as W
from oracle import step as S
from oracle.lattice import D2Q9, D3Q19
from oracle.coeffs import equal_sigma


def test_couette_profile_is_exact():
    nx, ny, U = 6, 10, 1e-3
    N = 2
    C0 = np.zeros((N, 1, ny, nx))
    C0[0] = 1.0
    par = S.Params(D2Q9, (nx, ny, 1), equal_sigma(N, 0.005), np.ones(N), m=0.05,
                   walls=(False, True, False),
                   open_faces={3: ((U, 0.0, 0.0), (1.0, 0.0))})
    f, g = S.initial_state(par, C0)
    for _ in range(2500):          # slowest mode decays as exp(-nu (pi/ny)^2 t): e^-41
        f, g, mac = S.step(f, g, par)
    mac = S.macroscopic(f, g, par)
    u = mac["v"][0, 0, :, 0]
    y = np.arange(ny) + 0.5
    assert np.abs(u - U * y / ny).max() <= 1e-10 * U
    assert np.abs(mac["v"][1]).max() <= 1e-12 * U
    # the face's equilibrium is at v_b, the node's at v: C is nudged near the
    # face and relaxes back on the Cahn-Hilliard time scale (2.5e-8 here,
    # 6e-11 after 12000 steps)
    assert np.abs(mac["C"][0] - 1.0).max() <= 1e-6


@pytest.mark.parametrize("lat,shape", [("D2Q9", (12, 7, 1)), ("D3Q19", (8, 5, 4))])
def test_plug_flow_is_a_fixed_point(lat, shape):
    L = D2Q9 if lat == "D2Q9" else D3Q19
    N = 3
    sig = equal_sigma(N, 0.005)
    sig[0, 2] = sig[2, 0] = 0.007
    Cb = np.array([0.5, 0.3, 0.2])
    u = np.array([2e-3, 0.0, 0.0])
    par = S.Params(L, shape, sig, np.ones(N), m=0.05, walls=(True, False, False),
                   open_faces={0: (u, Cb), 1: (u, Cb)})
    grid = (shape[2], shape[1], shape[0])
    C0 = np.broadcast_to(Cb.reshape(N, 1, 1, 1), (N,) + grid).copy()
    v0 = np.broadcast_to(u.reshape(3, 1, 1, 1), (3,) + grid).copy()
    f, g = S.initial_state(par, C0, v0)
    for _ in range(40):
        f, g, _ = S.step(f, g, par)
    mac = S.macroscopic(f, g, par)
    assert np.abs(mac["C"] - C0).max() <= 1e-14
    assert np.abs(mac["v"] - v0).max() <= 1e-14 * np.abs(u).max() * 1e3


def test_closed_open_faces_keep_mass():
    w = W.noise("D2Q9", (20, 12, 1), 3, amp=0.1, seed=3, sigma=0.006, m=0.05)
    N = 3
    mean = w["C0"].mean(axis=(1, 2, 3))
    # faces at rest whose boundary values equal the mean mixture: the mixture
    # only redistributes, mass exchange with the faces stays small
    par = S.Params(D2Q9, w["shape"], w["sigma"], w["tau"], m=w["m"], walls=(True, False, False),
                   open_faces={0: ((0, 0, 0), mean), 1: ((0, 0, 0), mean)})
    f, g = S.initial_state(par, w["C0"])
    m0 = S.concentrations(g, par).sum(axis=(1, 2, 3))
    for _ in range(100):
        f, g, mac = S.step(f, g, par)
    C = S.concentrations(g, par)
    assert np.abs(C.sum(axis=0) - 1.0).max() <= 1e-13
    assert np.abs(C.sum(axis=(1, 2, 3)) - m0).max() <= 5e-3 * m0.max()
    assert np.abs(mac["v"]).max() < 1e-3


def _pulse_run(nx, outlet, steps=120, ny=6, u=0.02):
    N = 2
    C0 = np.zeros((N, 1, ny, nx))
    C0[0] = 1.0
    x = np.arange(nx)
    v0 = np.zeros((3, 1, ny, nx))
    v0[0] = u + 0.002 * np.exp(-((x - 20) / 3.0) ** 2)[None, None, :]
    faces = {0: ((u, 0.0, 0.0), (1.0, 0.0))}
    kw = {}
    if outlet == "outflow":
        kw["outflow"] = 1
    elif outlet == "dirichlet":
        faces[1] = ((u, 0.0, 0.0), (1.0, 0.0))
    par = S.Params(D2Q9, (nx, ny, 1), equal_sigma(N, 0.005), np.ones(N), m=0.05,
                   walls=(True, False, False), open_faces=faces, **kw)
    f, g = S.initial_state(par, C0, v0)
    for _ in range(steps):
        f, g, _ = S.step(f, g, par)
    return S.macroscopic(f, g, par)["v"][0, 0, 0]


def test_convective_outflow_lets_a_pulse_leave():
    """A velocity pulse carried by a plug flow (inlet u = 0.02 on x-) passes
    the outlet of a 60-node channel.  Against the same run on a 240-node
    channel (outlet far away) the convective outflow (Eq. convect) leaves the
    flow within 5 % of the pulse amplitude, at least four times closer than a
    velocity-Dirichlet outlet, which reflects the pulse."""
    ref = _pulse_run(240, "dirichlet")[:60]
    d_out = np.abs(_pulse_run(60, "outflow") - ref).max()
    d_dir = np.abs(_pulse_run(60, "dirichlet") - ref).max()
    assert d_out < 0.05 * 0.002
    assert d_out < 0.25 * d_dir


@pytest.mark.parametrize("lat,shape", [("D2Q9", (14, 5, 1)), ("D3Q19", (9, 4, 5))])
def test_inlet_outflow_plug_flow_is_a_fixed_point(lat, shape):
    L = D2Q9 if lat == "D2Q9" else D3Q19
    N = 3
    Cb = np.array([0.5, 0.3, 0.2])
    u = np.array([3e-3, 0.0, 0.0])
    par = S.Params(L, shape, equal_sigma(N, 0.005), np.ones(N), m=0.05, walls=(True, False, False),
                   open_faces={0: (u, Cb)}, outflow=1)
    grid = (shape[2], shape[1], shape[0])
    C0 = np.broadcast_to(Cb.reshape(N, 1, 1, 1), (N,) + grid).copy()
    v0 = np.broadcast_to(u.reshape(3, 1, 1, 1), (3,) + grid).copy()
    f, g = S.initial_state(par, C0, v0)
    for _ in range(40):
        f, g, _ = S.step(f, g, par)
    mac = S.macroscopic(f, g, par)
    assert np.abs(mac["C"] - C0).max() <= 1e-13
    assert np.abs(mac["v"] - v0).max() <= 1e-14
    assert abs(par.outflow_state["U"] - u[0]) <= 1e-15


def test_outflow_mirror_symmetry():
    """Inlet on x- and outflow on x+, against the same run mirrored in x:
    C(x) and v_x(x) of the first equal C(nx-1-x) and -v_x(nx-1-x) of the
    second to rounding (a wrong sign of the outward normal or a wrong plane
    of the x- face breaks the symmetry at O(1))."""
    nx, ny, N = 20, 7, 3
    w = W.noise("D2Q9", (nx, ny, 1), N, amp=0.1, seed=12, sigma=0.006, m=0.05)
    Cb = np.array([0.6, 0.3, 0.1])
    u = 3e-3
    runs = []
    for inlet, out, sign in ((0, 1, 1.0), (1, 0, -1.0)):
        C0 = w["C0"] if sign > 0 else w["C0"][..., ::-1].copy()
        par = S.Params(D2Q9, (nx, ny, 1), w["sigma"], w["tau"], m=w["m"], walls=(True, False, False),
                       open_faces={inlet: (np.array([sign * u, 0.0, 0.0]), Cb)}, outflow=out)
        f, g = S.initial_state(par, C0)
        for _ in range(80):
            f, g, _ = S.step(f, g, par)
        mac = S.macroscopic(f, g, par)
        runs.append((mac["C"], mac["v"], par.outflow_state["U"]))
    (C1, v1, U1), (C2, v2, U2) = runs
    assert U1 > 1e-3 and abs(U1 - U2) <= 1e-15
    assert np.abs(C1 - C2[..., ::-1]).max() <= 1e-13
    assert np.abs(v1[0] - (-v2[0][..., ::-1])).max() <= 1e-13 * np.abs(v1[0]).max()
    assert np.abs(v1[1] - v2[1][..., ::-1]).max() <= 1e-13 * np.abs(v1[0]).max()
