"""Pins of the oracle's solid geometry (Sec. III C) on the CPU.

  face equivalence   solid rows (planes) that close a periodic axis give the
                     same trajectory as wall faces on the inner lattice: the
                     general solid mask reduces to the pinned face walls
  brute force        vectorised step == node-by-node loop with an irregular
                     obstacle, walls and TRT
  conservation       per-component mass with obstacles, for the constant and
                     the concentration-dependent mobility; solid nodes hold no
                     fluid (every field exactly 0 there)
"""
import numpy as np
import pytest

import workloads as W
from oracle import diag, naive
from oracle import step as S
from oracle.lattice import D2Q9, D3Q19


def params_of(w, **kw):
    lat = D2Q9 if w["lattice"] == "D2Q9" else D3Q19
    args = dict(D=w["D"], omega_stab=w["omega_stab"], trt_magic=w["trt_magic"],
                tau_g=w["tau_g"], m=w["m"], body_force=w["body_force"], walls=w["walls"])
    args.update(kw)
    return S.Params(lat, w["shape"], w["sigma"], w["tau"], **args)


def blob(shape, seed):
    """An irregular solid region: a disc plus two posts, in lattice order [nz, ny, nx]."""
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    rng = np.random.default_rng(seed)
    cx, cy = rng.uniform(0.3, 0.7) * nx, rng.uniform(0.3, 0.7) * ny
    s = (x - cx) ** 2 + (y - cy) ** 2 < (0.18 * min(nx, ny)) ** 2
    s |= (x == 1) & (y < ny // 3)
    s |= (x >= nx - 3) & (x <= nx - 2) & (y >= ny - 3)
    return s


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_solid_planes_equal_wall_faces(lat):
    if lat == "D2Q9":
        inner, axis = (20, 14, 1), 1
    else:
        inner, axis = (8, 7, 10), 2
    w = W.noise(lat, inner, 3, amp=0.2, seed=12)
    walls = [False, False, False]
    walls[axis] = True
    w.update(walls=tuple(walls), trt_magic=3.0 / 16.0, body_force=(3e-5, 1e-5, 0.0),
             tau=np.array([0.6, 1.0, 1.3]))
    pw = params_of(w)
    # the same fluid with one solid layer on each side of the closed axis, periodic
    padded = list(inner)
    padded[axis] += 2
    ax = 2 - axis                                    # array axis of lattice axis
    C0 = np.pad(w["C0"], [(0, 0)] + [(1, 1) if a == ax else (0, 0) for a in range(3)])
    solid = np.zeros((padded[2], padded[1], padded[0]), dtype=bool)
    idx = [slice(None)] * 3
    idx[ax] = 0
    solid[tuple(idx)] = True
    idx[ax] = -1
    solid[tuple(idx)] = True
    wp = dict(w, shape=tuple(padded), walls=(False, False, False), C0=C0)
    ps = params_of(wp, solid=solid)
    f1, g1 = S.initial_state(pw, w["C0"])
    f2, g2 = S.initial_state(ps, C0)
    for _ in range(60):
        f1, g1, _ = S.step(f1, g1, pw)
        f2, g2, _ = S.step(f2, g2, ps)
    inner_sl = [slice(None)] * 3
    inner_sl[ax] = slice(1, -1)
    sl = (Ellipsis,) + tuple(inner_sl)
    assert np.abs(f2[sl][1:] - f1[1:]).max() <= 1e-15 * np.abs(f1).max()
    assert np.abs(g2[sl] - g1).max() <= 1e-15 * np.abs(g1).max()
    assert np.all(f2[..., solid] == 0.0) and np.all(g2[..., solid] == 0.0)


def test_vectorised_equals_node_loop_with_obstacle():
    w = W.noise("D2Q9", (12, 10, 1), 3, amp=0.2, seed=5)
    w.update(walls=(False, True, False), trt_magic=3.0 / 16.0, body_force=(1e-4, -2e-5, 0.0),
             tau=np.array([0.6, 0.9, 1.3]))
    par = params_of(w, solid=blob(w["shape"], 1))
    f, g = S.initial_state(par, w["C0"])
    for _ in range(2):
        f, g, _ = S.step(f, g, par)
    f1, g1, _ = S.step(f, g, par)
    f2, g2 = naive.step(f, g, par)
    assert np.abs(f1[1:] - f2[1:]).max() <= 1e-12 * np.abs(f1).max()
    assert np.abs(g1 - g2).max() <= 1e-13 * np.abs(g1).max()


@pytest.mark.parametrize("mobility", ["constant", "c2c2"])
def test_mass_with_obstacles(mobility):
    w = W.noise("D2Q9", (40, 32, 1), 3, amp=0.1, seed=7)
    w.update(walls=(False, True, False), body_force=(1e-5, 0.0, 0.0))
    solid = blob(w["shape"], 3)
    par = params_of(w, solid=solid, mobility=mobility, m_star=10.0)
    f, g = S.initial_state(par, w["C0"])
    d0 = diag.diagnostics(f, g, par)
    for _ in range(200):
        f, g, mac = S.step(f, g, par)
    d1 = diag.diagnostics(f, g, par)
    for a, b in zip(d0["mass"], d1["mass"]):
        assert abs(b - a) <= 1e-13 * a
    C = S.concentrations(g, par)
    assert np.all(C[:, solid] == 0.0)
    assert np.abs(C.sum(axis=0)[~solid] - 1.0).max() <= 1e-14
    assert np.abs(C - S.concentrations(S.initial_state(par, w["C0"])[1], par)).max() > 1e-4
