"""Seeded synthetic inputs shared by the oracle tests, the HIP parity tests and
the benchmark.

This module only draws random numbers and builds initial shapes (tanh-smoothed
bands, discs and layers); it contains none of the lattice Boltzmann method's
arithmetic.  Every workload returns a plain dict describing one simulation:

  lattice      "D2Q9" or "D3Q19"
  shape        (nx, ny, nz)
  walls        (wx, wy, wz) booleans: halfway bounce-back on both faces of that axis
  sigma        N x N pairwise surface tensions
  tau          N hydrodynamic relaxation times (viscosity of the majority fluid)
  tau_g        N Cahn-Hilliard relaxation times
  m            mobility parameter of the concentration equilibrium
  D            interface width
  omega_stab   Omega of the stabilising term
  trt_magic    Lambda^TRT (0 selects BGK)
  body_force   (Fx, Fy, Fz)
  C0           [N, nz, ny, nx] float64 initial concentrations
  v0           [3, nz, ny, nx] float64 initial velocity or None (rest)

Interfaces are smoothed as 1/2 [1 + tanh(d/2)], d the signed distance in
lattice units ("tanh profiles of width 2").
"""
import numpy as np


def _smooth(d):
    return 0.5 * (1.0 + np.tanh(d / 2.0))


def _equal_sigma(N, s):
    return s * (np.ones((N, N)) - np.eye(N))


def _base(lattice, shape, sigma, tau, m, **kw):
    N = sigma.shape[0]
    out = dict(lattice=lattice, shape=tuple(int(s) for s in shape),
               walls=(False, False, False), sigma=np.asarray(sigma, dtype=np.float64),
               tau=np.full(N, float(tau)) if np.isscalar(tau) else np.asarray(tau, float),
               tau_g=np.ones(N), m=float(m), D=4.0, omega_stab=0.0, trt_magic=0.0,
               body_force=(0.0, 0.0, 0.0), v0=None)
    out.update(kw)
    return out


def lens_2d(nx=64, ny=64, radius=12.0, sigma=None, m=0.05, tau=1.0):
    """Liquid lens: fluid 1 fills the lower half (y < ny/2), fluid 2 the upper
    half, and a disc of fluid 3 is centred on the middle interface.  The domain
    is periodic, so a second flat 1|2 interface sits at y = 0."""
    if sigma is None:
        sigma = _equal_sigma(3, 0.005)
    j = np.arange(ny, dtype=np.float64)[:, None]
    i = np.arange(nx, dtype=np.float64)[None, :]
    half = ny / 2.0
    yc = half - 0.5                       # the middle interface, between rows
    band_centre = half / 2.0 - 0.5        # centre of fluid 1's band
    dist = ((j - band_centre + half) % ny) - half
    d_band = half / 2.0 - np.abs(dist)
    c1r = _smooth(d_band) * np.ones((ny, nx))
    r = np.sqrt((i - (nx / 2.0 - 0.5)) ** 2 + (j - yc) ** 2)
    c3 = _smooth(-(r - radius) * 1.0)
    c1 = (1 - c3) * c1r
    c2 = (1 - c3) * (1 - c1r)
    C0 = np.stack([c1, c2, c3])[:, None, :, :]
    return _base("D2Q9", (nx, ny, 1), sigma, tau, m, C0=C0, name="lens_2d",
                 y_interface=yc)


def table1_lens(s, nx=300, ny=150, radius=35.0, m=0.05, ncomp=6):
    """Four-fluid lens of Table I inside an N = 6 model (Sec. IV A): fluid 1
    fills the lower band and fluid 2 the upper (periodic), a disc of radius R
    centred on the middle 1|2 interface holds fluid 3 in its left half and
    fluid 4 in its right half, and fluids 5, 6 are exactly 0.  sigma_12 =
    0.005, sigma_13 = sigma_14 = sigma_23 = sigma_24 = sigma_34 = s, and every
    tension of fluids 5, 6 is 0.005.  tau = 1 (eta = 1/6), tau_g = 1."""
    j = np.arange(ny, dtype=np.float64)[:, None]
    i = np.arange(nx, dtype=np.float64)[None, :]
    half = ny / 2.0
    yc = half - 0.5
    xc = nx / 2.0 - 0.5
    band_centre = half / 2.0 - 0.5
    dist = ((j - band_centre + half) % ny) - half
    c1r = _smooth(half / 2.0 - np.abs(dist)) * np.ones((ny, nx))
    disc = _smooth(-(np.sqrt((i - xc) ** 2 + (j - yc) ** 2) - radius))
    right = _smooth(i - xc) * np.ones((ny, nx))
    c3 = disc * (1 - right)
    c4 = disc * right
    c1 = (1 - disc) * c1r
    c2 = (1 - disc) * (1 - c1r)
    zero = np.zeros((ny, nx))
    C0 = np.stack([c1, c2, c3, c4] + [zero] * (ncomp - 4))[:, None, :, :]
    sigma = np.full((ncomp, ncomp), 0.005)
    for a in range(4):
        for b in range(4):
            sigma[a, b] = s
    sigma[0, 1] = sigma[1, 0] = 0.005
    np.fill_diagonal(sigma, 0.0)
    return _base("D2Q9", (nx, ny, 1), sigma, 1.0, m, C0=C0, name="table1_lens", y_interface=yc)


def janus_2d(nx=100, ny=100, radius=20.0, offset=25.0, sigma=None, m=0.05, tau=1.0,
             ncomp=4):
    """Janus droplet (Sec. IV A): a disc of fluid 2 at the centre and discs of
    fluids 3 and 4 offset to the right and to the left, each minus what it
    shares with the discs placed before it; fluid 1 fills the rest.  Default
    tensions: sigma_14 = sigma_24 = 0.0095, all others 0.005."""
    if sigma is None:
        sigma = _equal_sigma(max(ncomp, 4), 0.005)
        sigma[0, 3] = sigma[3, 0] = 0.0095
        sigma[1, 3] = sigma[3, 1] = 0.0095
        sigma = sigma[:ncomp, :ncomp]
    j = np.arange(ny, dtype=np.float64)[:, None]
    i = np.arange(nx, dtype=np.float64)[None, :]
    cx, cy = nx / 2.0 - 0.5, ny / 2.0 - 0.5

    def disc(x0):
        return _smooth(-(np.sqrt((i - x0) ** 2 + (j - cy) ** 2) - radius))

    d2 = disc(cx)
    d3 = disc(cx + offset) * (1 - d2)
    d4 = disc(cx - offset) * (1 - d2) * (1 - disc(cx + offset))
    c1 = 1 - d2 - d3 - d4
    comps = [c1, d2, d3, d4][:ncomp] + [np.zeros_like(c1)] * max(0, ncomp - 4)
    C0 = np.stack(comps)[:, None, :, :]
    return _base("D2Q9", (nx, ny, 1), sigma, tau, m, C0=C0, name="janus_2d")


def droplet_2d(nx=48, ny=48, radius=10.0, sigma12=0.005, m=0.05, tau=1.0, ncomp=2):
    """A disc of fluid 2 in fluid 1 (further components absent)."""
    sigma = _equal_sigma(ncomp, sigma12)
    j = np.arange(ny, dtype=np.float64)[:, None]
    i = np.arange(nx, dtype=np.float64)[None, :]
    c2 = _smooth(-(np.sqrt((i - nx / 2 + 0.5) ** 2 + (j - ny / 2 + 0.5) ** 2) - radius))
    comps = [1 - c2, c2] + [np.zeros_like(c2)] * (ncomp - 2)
    C0 = np.stack(comps)[:, None, :, :]
    return _base("D2Q9", (nx, ny, 1), sigma, tau, m, C0=C0, name="droplet_2d")


def noise(lattice, shape, ncomp_present, ncomp_total=None, amp=0.02, seed=0,
          sigma=0.01, m=0.1, tau=1.0):
    """Uniform mixture 1/P + U(-amp, amp) for P present components, renormalised to
    sum 1; further components are exactly 0.  P = 4 and mean 0.25 reproduce the
    quaternary phase-separation inputs."""
    ncomp_total = ncomp_total or ncomp_present
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    C = 1.0 / ncomp_present + rng.uniform(-amp, amp, size=(ncomp_present, nz, ny, nx))
    C /= C.sum(axis=0, keepdims=True)
    if ncomp_total > ncomp_present:
        C = np.concatenate([C, np.zeros((ncomp_total - ncomp_present, nz, ny, nx))])
    return _base(lattice, shape, _equal_sigma(ncomp_total, sigma), tau, m, C0=C,
                 name=f"noise_{lattice}_{ncomp_present}of{ncomp_total}")


def coarsening_2d(n=400, ncomp=4, seed=0, sigma=0.005, m=0.1):
    """Phase separation from the recipe of Sec. IV B: every C_i drawn from
    U[0, 2/N] at each node, then normalised to sum 1; all sigma equal, eta =
    1/6 (tau = 1), tau_g = 1."""
    rng = np.random.default_rng(seed)
    C = rng.uniform(0.0, 2.0 / ncomp, size=(ncomp, 1, n, n))
    C /= C.sum(axis=0, keepdims=True)
    return _base("D2Q9", (n, n, 1), _equal_sigma(ncomp, sigma), 1.0, m, C0=C, name="coarsening_2d")


def quaternary_2d(n=512, seed=0):
    """D2Q9, N = 4, n x n periodic, 0.25 + U(-0.02, 0.02) renormalised;
    sigma = 0.01, tau = tau_g = 1, m = 0.1."""
    return noise("D2Q9", (n, n, 1), 4, seed=seed)


def quaternary_3d(n=256, seed=0, with_absent=True, nz=None):
    """D3Q19, N = 4 (+ a fifth component that is exactly 0), n^3 periodic,
    0.25 + U(-0.02, 0.02) renormalised; sigma = 0.01, tau = tau_g = 1, m = 0.1."""
    nz = nz or n
    return noise("D3Q19", (n, n, nz), 4, 5 if with_absent else 4, seed=seed)


def layered_3d(nx=16, ny=16, nz=192, nlayers=6, tau_lo=0.6, tau_hi=1.5, force=1e-7,
               sigma=0.005, m=1.0 / 50.0, trt_magic=3.0 / 16.0, v0_profile=None):
    """Layered channel between halfway bounce-back walls on the z faces.  Layer n
    fills z in [L(n-1), L n) with L = nz / nlayers; node j sits at z = j + 1/2.
    Relaxation times linearly spaced from tau_lo to tau_hi.  v0_profile, if
    given, is a length-nz array of u_x(z) used as the initial velocity."""
    L = nz / nlayers
    z = np.arange(nz, dtype=np.float64) + 0.5
    # above[q] is the smoothed indicator of z > L q; layer q (0-based, bottom
    # first) is above[q] - above[q+1], and the layers telescope to 1.
    above = [np.ones(nz)] + [_smooth(z - L * q) for q in range(1, nlayers)] + [np.zeros(nz)]
    layers = [above[q] - above[q + 1] for q in range(nlayers)]
    C = np.stack(layers)
    C = np.clip(C, 0.0, None)
    C /= C.sum(axis=0, keepdims=True)
    C0 = np.broadcast_to(C[:, :, None, None], (nlayers, nz, ny, nx)).copy()
    tau = np.linspace(tau_lo, tau_hi, nlayers)
    out = _base("D3Q19", (nx, ny, nz), _equal_sigma(nlayers, sigma), tau, m, C0=C0,
                walls=(False, False, True), trt_magic=trt_magic,
                body_force=(force, 0.0, 0.0), name="layered_3d")
    if v0_profile is not None:
        v0 = np.zeros((3, nz, ny, nx))
        v0[0] = np.asarray(v0_profile, dtype=np.float64)[:, None, None]
        out["v0"] = v0
    out["layer_edges"] = [L * q for q in range(nlayers + 1)]
    return out


def spreading_omega(sigma):
    """Omega = 0 when every spreading parameter S_ij;k = s_ij - s_ik - s_jk is
    negative, else 1/18 (the value used for the emulsion application)."""
    N = sigma.shape[0]
    for a in range(N):
        for b in range(a + 1, N):
            for c in range(N):
                if c not in (a, b) and sigma[a, b] - sigma[a, c] - sigma[b, c] > 0:
                    return 1.0 / 18.0
    return 0.0


def batch_members(count=256, seed=0, sides=None):
    """Independent D2Q9, N = 3 lens / Janus problems of uneven sizes.

    Side L in {64, 96, ..., 512}; sigma_12 = 0.005, sigma_13 and sigma_23 drawn
    from U[0.0025, 0.01]; type 0 = lens (config of lens_2d scaled to
    R = 0.1875 L), type 1 = Janus (two half discs of fluids 2 and 3, R = 0.2 L,
    centred in fluid 1).  tau = tau_g = 1, m = 0.05, Omega from the spreading
    parameters."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        L = 64 + 32 * int(rng.integers(0, 15)) if sides is None else int(sides[b])
        s13, s23 = rng.uniform(0.0025, 0.01, size=2)
        kind = int(rng.integers(0, 2))
        sigma = np.array([[0, 0.005, s13], [0.005, 0, s23], [s13, s23, 0]], dtype=np.float64)
        if kind == 0:
            w = lens_2d(L, L, radius=0.1875 * L, sigma=sigma, m=0.05)
        else:
            j = np.arange(L, dtype=np.float64)[:, None]
            i = np.arange(L, dtype=np.float64)[None, :]
            c = L / 2.0 - 0.5
            disc = _smooth(-(np.sqrt((i - c) ** 2 + (j - c) ** 2) - 0.2 * L))
            right = _smooth(i - c)
            c2 = disc * (1 - right)
            c3 = disc * right
            C0 = np.stack([1 - disc, c2, c3])[:, None, :, :]
            w = _base("D2Q9", (L, L, 1), sigma, 1.0, 0.05, C0=C0, name="janus_half_2d")
        w["omega_stab"] = spreading_omega(sigma)
        w["kind"] = kind
        out.append(w)
    return out


def ulp_perturbed(C0, seed=20261203):
    """C0 with every nonzero value moved by one unit in the last place, up or
    down by a seeded coin (zeros stay exactly 0).  Parity tests run a case
    from C0 and from this input: how far the two results drift apart measures
    how strongly the problem amplifies rounding-sized differences, which
    bounds how closely two correct implementations that round differently
    can agree."""
    C0 = np.asarray(C0, dtype=np.float64)
    rng = np.random.default_rng(seed)
    up = rng.integers(0, 2, size=C0.shape).astype(bool)
    moved = np.where(up, np.nextafter(C0, np.inf), np.nextafter(C0, -np.inf))
    return np.where(C0 == 0.0, C0, moved)


def tjunction(lattice="D2Q9", nx=48, ny=24, nz=1, channel=12, branch=(14, 22), u_main=3e-3,
              u_side=2e-3, ncomp=3, amp=0.0, seed=0, sigma=0.005, m=0.05, omega_stab=0.0):
    """A T-junction in the style of the emulsion device of Sec. V B: a main
    channel y < channel along x with an inlet of pure fluid 1 on x- (velocity
    u_main along +x) and the convective outflow on x+; a side branch of
    columns branch[0] <= x < branch[1] rising to the y+ face, where pure fluid
    2 enters at u_side along -y.  Solid nodes fill y >= channel outside the
    branch (they meet both open faces and the outflow at the domain's
    corners); y- is a wall face.  The main channel starts filled with fluid 3
    (amp > 0: a seeded uniform mixture 1/N + U(-amp, amp) renormalised
    instead).  Returns the workload dict plus "solid" [nz, ny, nx], "faces"
    {face: (v_b, C_b)} and "outflow" (the face index).  In D3Q19 the layout
    is extruded along z (periodic)."""
    N = ncomp
    shape = (nx, ny, nz)
    w = _base(lattice, shape, _equal_sigma(N, sigma), 1.0, m, omega_stab=omega_stab)
    w["walls"] = (True, True, False)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    solid = (y >= channel) & ((x < branch[0]) | (x >= branch[1]))
    C0 = np.zeros((N, nz, ny, nx))
    if amp > 0.0:
        rng = np.random.default_rng(seed)
        C0 = 1.0 / N + rng.uniform(-amp, amp, size=C0.shape)
        C0 /= C0.sum(axis=0, keepdims=True)
    else:
        C0[min(2, N - 1)] = 1.0
    C0[:, solid] = 0.0
    Cin = np.zeros(N)
    Cin[0] = 1.0
    Cside = np.zeros(N)
    Cside[min(1, N - 1)] = 1.0
    w.update(C0=C0, name=f"tjunction_{lattice}_{nx}x{ny}x{nz}", solid=solid,
             faces={0: ((u_main, 0.0, 0.0), Cin), 3: ((0.0, -u_side, 0.0), Cside)}, outflow=1)
    return w
