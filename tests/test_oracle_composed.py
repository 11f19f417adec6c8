"""Pins of the oracle's open faces and convective outflow together with solid
nodes (Sec. III C; the emulsion device of Sec. V B combines all three).

  face equivalence   a channel whose side walls are solid layers, with an
                     inlet on x- and the convective outflow on x+, gives the
                     same trajectory as the channel with wall faces: at the
                     corners where a wall face beats an open face, the solid
                     layer continued beyond the open face (a link whose in-face
                     part leads to a solid node is a wall link) must act the
                     same, and the outflow's mean velocity must skip the solid
                     nodes of the plane
  brute force        vectorised step == the node-by-node loop (independent
                     index arithmetic for walls, solids, open faces and their
                     corners) on a T-junction with two inlets and walls, in
                     D2Q9 and D3Q19
  refusal            an outflow plane whose solid nodes do not continue into
                     the plane inside it is refused
"""
import numpy as np
import pytest

import workloads as W
from oracle import naive
from oracle import step as S
from oracle.lattice import D2Q9, D3Q19


def _params(w, **kw):
    lat = D2Q9 if w["lattice"] == "D2Q9" else D3Q19
    args = dict(D=w["D"], omega_stab=w["omega_stab"], trt_magic=w["trt_magic"],
                tau_g=w["tau_g"], m=w["m"], body_force=w["body_force"], walls=w["walls"])
    args.update(kw)
    return S.Params(lat, w["shape"], w["sigma"], w["tau"], **args)


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_solid_side_walls_equal_wall_faces_with_inlet_and_outflow(lat):
    if lat == "D2Q9":
        inner = (18, 9, 1)
    else:
        inner = (10, 6, 4)
    w = W.noise(lat, inner, 3, amp=0.15, seed=21, sigma=0.006, m=0.05)
    w.update(tau=np.array([0.7, 1.0, 1.2]), trt_magic=3.0 / 16.0)
    Cb = np.array([0.55, 0.3, 0.15])
    u = np.array([4e-3, 1e-3, 0.0])
    faces = {0: (u, Cb)}
    # (a) wall faces on y
    pa = _params(dict(w, walls=(True, True, False)), open_faces=faces, outflow=1)
    # (b) y periodic, one solid layer below and above the fluid rows
    nx, ny, nz = inner
    C0b = np.pad(w["C0"], [(0, 0), (0, 0), (1, 1), (0, 0)])
    solid = np.zeros((nz, ny + 2, nx), dtype=bool)
    solid[:, 0] = solid[:, -1] = True
    wb = dict(w, shape=(nx, ny + 2, nz), walls=(True, False, False))
    pb = _params(wb, open_faces=faces, outflow=1, solid=solid)
    fa, ga = S.initial_state(pa, w["C0"])
    fb, gb = S.initial_state(pb, C0b)
    for _ in range(50):
        fa, ga, _ = S.step(fa, ga, pa)
        fb, gb, _ = S.step(fb, gb, pb)
    sl = (Ellipsis, slice(None), slice(1, -1), slice(None))
    assert pa.outflow_state["U"] > 1e-3
    assert abs(pa.outflow_state["U"] - pb.outflow_state["U"]) <= 1e-17
    assert np.abs(fb[sl][1:] - fa[1:]).max() <= 1e-15 * np.abs(fa).max()
    assert np.abs(gb[sl] - ga).max() <= 1e-15 * np.abs(ga).max()
    assert np.all(fb[..., solid] == 0.0) and np.all(gb[..., solid] == 0.0)
    # a flowing channel (the corners carry momentum)
    ma = S.macroscopic(fa, ga, pa)
    assert np.abs(ma["v"][0]).max() > 1e-3


@pytest.mark.parametrize("lat,shape", [("D2Q9", (12, 9, 1)), ("D3Q19", (9, 7, 3))])
def test_tjunction_node_loop(lat, shape):
    nx, ny, nz = shape
    w = W.tjunction(lat, nx=nx, ny=ny, nz=nz, channel=5, branch=(4, 7), amp=0.15, seed=4)
    w.update(tau=np.array([0.7, 1.0, 1.3]), trt_magic=3.0 / 16.0, body_force=(2e-5, -1e-5, 0.0))
    faces = dict(w["faces"])
    faces[1] = ((3e-3, 0.0, 0.0), np.array([0.2, 0.3, 0.5]))     # a second inlet instead of the outflow
    par = _params(w, open_faces=faces, solid=w["solid"])
    f, g = S.initial_state(par, w["C0"])
    for _ in range(3):
        f, g, _ = S.step(f, g, par)
    f1, g1, _ = S.step(f, g, par)
    f2, g2 = naive.step(f, g, par)
    assert np.abs(f1[1:] - f2[1:]).max() <= 1e-12 * np.abs(f1).max()
    assert np.abs(g1 - g2).max() <= 1e-13 * np.abs(g1).max()
    # the prism rule is exercised: links of fluid nodes on the y+ face whose
    # in-face part leads into the solid block
    e = D2Q9.e[5] if lat == "D2Q9" else D3Q19.e[7]           # (1, 1, 0)
    m = S.open_face_masks(par, e)
    assert 3 in m and not m[3][..., ny - 1, 6].any()          # x = 6 -> x + 1 = 7 is solid
    assert m[3][..., ny - 1, 5].all()


def test_outflow_plane_solids_must_continue():
    w = W.tjunction(nx=16, ny=10, channel=5, branch=(4, 7))
    solid = w["solid"].copy()
    solid[0, 2, -1] = True                                    # a solid node on plane N only
    with pytest.raises(ValueError):
        _params(w, open_faces=w["faces"], outflow=1, solid=solid)
    _params(w, open_faces=w["faces"], outflow=1, solid=w["solid"])
