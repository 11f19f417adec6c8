"""One time step of the N-component free-energy LBM, vectorised over the
lattice with NumPy in FP64.  Test infrastructure only.

State (post-streaming, time t):
  f[Q, nz, ny, nx]      hydrodynamic populations (Sec. III A)
  g[N, Q, nz, ny, nx]   one population set per component (Sec. III B)

Order of one step (the paper gives no pseudo-code; this is the order in which
each quantity is defined in terms of the previous ones):
  1. C_i = sum_k g_{i,k}                                   (zeroth moment of g)
  2. E_B(C) pointwise                                      (Eq. FreeEnergy)
  3. grad C_i, lap C_i, grad E_B with the isotropic stencils (Eq. gradstencil
     and the Laplacian after it); a neighbour inside a wall is replaced by the
     centre value (last paragraph before the open-boundary conditions).
  4. mu~_i (factored form by default; see potential.py)
  5. F = grad E_B + sum_{i != j} kappa_ij lap C_j grad C_i + F_b   (Eq. Fsnew)
     or, as a negative control, F = sum_i mu_i grad C_i + F_b     (Eq. ststand)
  6. v = sum_k e_k f_k + F/2                               (Eq. nmom, rho = 1)
     P = c_s^2/(1-w_0) [sum_{k != 0} f_k + s_0(v)]          (Eq. pres, grad rho = 0)
  7. tau = tau_i of the component with the largest C (lowest index on ties);
     omega+ = 1/tau; omega- = omega+ (BGK) or from the magic parameter
     Lambda^TRT = (1/omega+ - 1/2)(1/omega- - 1/2).
  8. TRT collision of f towards f^eq (Eq. feq) with the forcing of Eqs. FTRT and
     hydroforce (grad rho = 0).
  9. BGK collision of g (Eq. glbe) towards g^eq.
 10. Streaming psi_k(x + e_k) <- psi*_k(x), periodic, or halfway bounce-back
     psi_kbar(x) <- psi*_k(x) when x + e_k is inside a wall.

Readings (where the printed text is garbled or silent):
  * N - 1 concentration LBEs are evolved and one component (``implicit``,
    default the last as in Sec. II) follows from sum_i C_i = 1 (text after
    Eq. CHFlux).  The slot of the implicit component in g stays zero.  Any
    component can be chosen; an absent component must not be the implicit one,
    because 1 - sum of the others is zero only to rounding.
  * f^eq_0 carries (P/c_s^2)(w_0 - 1) so that sum_k f^eq_k = 0.  f_0 is read by
    no other quantity (P sums k != 0, e_0 = 0, TRT pairs 0 with itself), so the
    choice affects only f_0 itself.
  * g^eq ("rest" form): g^eq_{i,0} = C_i (1 + s_0) + (1 - w_0) m mu~_i,
    g^eq_{i,k} = C_i s_k - w_k m mu~_i for k != 0.  Zeroth moment C_i, first
    moment C_i v, second moment C_i v v - c_s^2 m mu~_i I: the Cahn-Hilliard
    flux J_i = M grad mu~_i with M = c_s^2 m (tau_g - 1/2).  The "printed" option
    adds w_k C_i to every direction, which adds a Fickian c_s^2 C_i I to the
    second moment.
  * rho = 1 exactly (rho_i = 1 for every component), so grad rho terms vanish.
  * Concentration-dependent mobility (Appendix C, ``mobility="c2c2"``): the
    per-node alpha_ij = C_i^2 C_j^2, alpha_ii = -sum_{j != i} alpha_ij replaces
    the constant alpha inside the flux only.  g^eq takes m = 0 and every
    evolved g gains the source (1 - 1/(2 tau_g)) w_k m* e_k.G_i after its BGK
    relaxation, with G_i = sum_j alpha_ij grad(mu_j + phi_j + xi_j) from the
    same isotropic gradient stencil as every other gradient; the mobility is
    M = c_s^2 m* (tau_g - 1/2).  alpha_ij is evaluated with all N
    concentrations of the node (the implicit one included).
  * Open faces (Sec. III C, ``open_faces={face: (v_b, C_b)}``, face 0..5 =
    x-, x+, y-, y+, z-, z+ of a walled axis): a population entering across
    the face is the node's own opposite post-collision one plus 2 w_k
    (e_k . v_b) / c_s^2 for f (velocity Dirichlet, rho_b = 1; the sign that
    gives the fluid the face's momentum) and, for g, minus it plus
    g^eq_k + g^eq_kbar of (C_b, v_b) (anti-bounce-back with the even part of
    the equilibrium, which keeps a uniform state at the boundary values
    fixed).  mu~ in that equilibrium is the bulk value of the uniform state
    C_b.  Stencil neighbours beyond the face take the boundary values (C_b,
    E_B(C_b)).  Where a link crosses a wall face and an open face (a corner),
    the wall wins; where it crosses two open faces, the first axis's face.
    A solid node on an open face continues beyond it (a prism normal to the
    face): a link across the face whose in-face part leads to a solid node is
    a wall link (bounce-back, centre value), which makes solid layers along
    a channel behave at an inlet exactly as wall faces do.
  * Convective outflow (Sec. III C, Eq. convect, ``outflow=face`` of a walled
    axis): after streaming, every population (all k, f and g) of the boundary
    plane N becomes (q(N, t) + U q(N-1, t+1)) / (1 + U), q(N, t) the plane's
    post-streaming values of the previous step.  U is the mean over plane N-1
    of the populations' normal momentum sum_k (e_k . n) f_k after streaming
    (without the F/2 term, which would need the new state's stencils), and 0
    if that mean points inwards.  Stencil neighbours beyond the face take
    ghost values of C_i and E_B convected the same way, psi(N+1, t+1) =
    (psi(N+1, t) + U psi(N, t+1)) / (1 + U), starting at psi(N, 0).  The
    previous planes, U and the ghosts are state: they live in
    ``par.outflow_state`` (set by initial_state, advanced by step).  Solid
    nodes must continue straight through the outflow plane (the same on
    planes N and N-1); U is the mean over the fluid nodes of plane N-1, and
    solid nodes of plane N stay empty.
"""
import numpy as np

from . import potential
from .lattice import CS2


class Params:
    """Problem statement of one simulation (Sec. II-III)."""

    def __init__(self, lattice, shape, sigma, tau, *, D=4.0, omega_stab=0.0,
                 trt_magic=0.0, tau_g=None, m=0.02, body_force=(0.0, 0.0, 0.0),
                 walls=(False, False, False), mu_form="factored",
                 force_form="conservative", geq_form="rest", hydro=True,
                 implicit=None, mobility="constant", m_star=10.0, solid=None,
                 open_faces=None, outflow=None):
        from .coeffs import Coefficients
        self.lat = lattice
        nx, ny, nz = shape
        if lattice.dim == 2 and nz != 1:
            raise ValueError("D2Q9 needs nz == 1")
        self.shape = (nx, ny, nz)
        self.co = Coefficients(sigma, D)
        self.N = self.co.N
        self.tau = np.asarray(tau, dtype=np.float64).reshape(self.N)
        self.tau_g = (np.ones(self.N) if tau_g is None
                      else np.asarray(tau_g, dtype=np.float64).reshape(self.N))
        self.omega_stab = float(omega_stab)
        self.trt_magic = float(trt_magic)
        self.m = float(m)
        self.body_force = np.asarray(body_force, dtype=np.float64).reshape(3)
        self.walls = tuple(bool(w) for w in walls)
        self.mu_form = mu_form
        self.force_form = force_form
        self.geq_form = geq_form
        self.hydro = hydro
        if solid is None:
            self.solid = None
        else:
            self.solid = np.asarray(solid, dtype=bool).reshape(self.grid)
            if self.solid.all():
                raise ValueError("no fluid node")
        self.open_faces = {}
        for face, (vb, Cb) in (open_faces or {}).items():
            if not 0 <= face < 6 or not self.walls[face // 2]:
                raise ValueError("an open face must lie on a walled axis")
            self.open_faces[int(face)] = (np.asarray(vb, dtype=np.float64).reshape(3),
                                          np.asarray(Cb, dtype=np.float64).reshape(self.N))
        if self.open_faces and mobility != "constant":
            raise ValueError("open faces take no mobility variant")
        self.outflow = None if outflow is None else int(outflow)
        if self.outflow is not None:
            if not 0 <= self.outflow < 6 or not self.walls[self.outflow // 2]:
                raise ValueError("the outflow face must lie on a walled axis")
            if self.outflow in self.open_faces or mobility != "constant":
                raise ValueError("the outflow face takes no open face or mobility variant")
            if self.solid is not None:
                bn, inner = _plane(self), _plane(self, 1)
                if not np.array_equal(self.solid[bn[1:]], self.solid[inner[1:]]):
                    raise ValueError("solid nodes must continue straight through the outflow plane "
                                     "(the same on its plane and the plane inside it)")
        self.outflow_state = None
        if mobility not in ("constant", "c2c2"):
            raise ValueError(mobility)
        self.mobility = mobility
        self.m_star = float(m_star)
        self.implicit = self.N - 1 if implicit is None else int(implicit)
        if not 0 <= self.implicit < self.N:
            raise ValueError("implicit component out of range")
        self.evolved = [i for i in range(self.N) if i != self.implicit]

    @property
    def grid(self):
        nx, ny, nz = self.shape
        return (nz, ny, nx)


def _axis(a):
    """Array axis of lattice axis a (0 = x, 1 = y, 2 = z) for [..., nz, ny, nx]."""
    return -1 - a


def wall_mask(par, e):
    """True at nodes whose neighbour x + e lies inside a wall: beyond a wall
    face, or a solid node (Sec. III C: halfway bounce-back at every solid
    boundary, and the stencil takes psi(x) for a neighbour inside a solid)."""
    nz, ny, nx = par.grid
    mask = np.zeros((nz, ny, nx), dtype=bool)
    n = (nx, ny, nz)
    for a in range(3):
        if not par.walls[a] or e[a] == 0:
            continue
        idx = [slice(None)] * 3
        idx[_axis(a) + 3] = n[a] - 1 if e[a] > 0 else 0
        mask[tuple(idx)] = True
    if par.solid is not None:
        mask |= np.roll(par.solid, shift=(-int(e[2]), -int(e[1]), -int(e[0])), axis=(0, 1, 2))
    return mask


def open_face_masks(par, e):
    """{face: nodes whose link to x + e leaves across that open face}, with a
    wall face taking precedence and, between open faces, the first axis.
    With solid nodes, a solid node on the face continues beyond it: a link
    whose part along the face (e without its normal component) leads from x
    to a solid node inside the lattice is a wall link, not an open one."""
    out = {}
    faces = set(par.open_faces)
    if par.outflow is not None:
        faces.add(par.outflow)
    if not faces:
        return out
    nz, ny, nx = par.grid
    n = (nx, ny, nz)
    grid = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    idx = (grid[2], grid[1], grid[0])
    plain = np.zeros((nz, ny, nx), dtype=bool)
    decided = np.zeros((nz, ny, nx), dtype=bool)
    for a in range(3):
        if not par.walls[a] or e[a] == 0:
            continue
        face = 2 * a + (1 if e[a] > 0 else 0)
        cross = (idx[a] + int(e[a]) < 0) | (idx[a] + int(e[a]) >= n[a])
        if face in faces:
            m = cross & ~decided
            out[face] = out.get(face, np.zeros_like(m)) | m
            decided |= cross
        else:
            plain |= cross
    out = {f: m & ~plain for f, m in out.items()}
    if par.solid is not None:
        for f in out:
            et = [int(c) for c in e]
            et[f // 2] = 0
            if not any(et):
                continue
            # x + et inside the lattice (no face crossed) and solid
            inside = np.ones((nz, ny, nx), dtype=bool)
            for a in range(3):
                if et[a] != 0 and par.walls[a]:
                    inside &= (idx[a] + et[a] >= 0) & (idx[a] + et[a] < n[a])
            prism = inside & np.roll(par.solid, shift=(-et[2], -et[1], -et[0]), axis=(0, 1, 2))
            out[f] = out[f] & ~prism
    return out


def neighbour(psi, e, par, bvals=None):
    """psi(x + e) with periodic wrap, or psi(x) where x + e is inside a wall;
    beyond an open face the face's value bvals[face] when given."""
    out = np.roll(psi, shift=(-int(e[2]), -int(e[1]), -int(e[0])), axis=(-3, -2, -1))
    mask = wall_mask(par, e)
    if mask.any():
        out = np.where(mask, psi, out)
    if bvals is not None:
        for face, m in open_face_masks(par, e).items():
            if face in bvals:
                val = bvals[face]
                if np.ndim(val) > 0:      # a ghost plane: the value where the link lands
                    val = np.roll(val, shift=(-int(e[2]), -int(e[1]), -int(e[0])), axis=(-3, -2, -1))
                out = np.where(m, val, out)
    return out


def gradient(psi, par, bvals=None):
    """(1/c_s^2) sum_{k>=1} w_k e_k [psi(x+e_k) - psi(x)]  -> [3, ...]."""
    lat = par.lat
    out = np.zeros((3,) + psi.shape)
    for k in range(1, lat.Q):
        d = neighbour(psi, lat.e[k], par, bvals) - psi
        for a in range(3):
            if lat.e[k, a] != 0:
                out[a] = out[a] + lat.w[k] * lat.e[k, a] * d
    return out / CS2


def laplacian(psi, par, bvals=None):
    """(2/c_s^2) sum_{k>=1} w_k [psi(x+e_k) - psi(x)]."""
    lat = par.lat
    out = np.zeros(psi.shape)
    for k in range(1, lat.Q):
        out = out + lat.w[k] * (neighbour(psi, lat.e[k], par, bvals) - psi)
    return 2.0 * out / CS2


def s_k(lat, v):
    """s_k(v) = w_k [v.e_k/c_s^2 + (v.e_k)^2/(2c_s^4) - v.v/(2c_s^2)] -> [Q, ...]."""
    vv = (v * v).sum(axis=0)
    out = np.empty((lat.Q,) + v.shape[1:])
    for k in range(lat.Q):
        ev = sum(lat.e[k, a] * v[a] for a in range(3))
        out[k] = lat.w[k] * (ev / CS2 + ev * ev / (2 * CS2 * CS2) - vv / (2 * CS2))
    return out


def concentrations(g, par):
    """C_i = sum_k g_{i,k} for the evolved components; the implicit component
    is 1 minus the others, summed in increasing component order."""
    C = g.sum(axis=1)
    rest = np.zeros(C.shape[1:])
    for i in par.evolved:
        rest = rest + C[i]
    C[par.implicit] = 1.0 - rest
    if par.solid is not None:
        C[:, par.solid] = 0.0
    return C


def macroscopic(f, g, par):
    """Steps 1-7: every node quantity the collision needs, as a dict."""
    lat, co, N = par.lat, par.co, par.N
    C = concentrations(g, par)
    EB = potential.bulk_energy(C, co)
    bc = [None] * N
    beb = None
    if par.open_faces or par.outflow is not None:
        bc = [{f: Cb[i] for f, (vb, Cb) in par.open_faces.items()} for i in range(N)]
        beb = {f: float(potential.bulk_energy(Cb.reshape(N, 1), co)[0])
               for f, (vb, Cb) in par.open_faces.items()}
        if par.outflow is not None:
            st = par.outflow_state
            for i in range(N):
                bc[i][par.outflow] = _plane_field(par, st["ghost_C"][i])
            beb[par.outflow] = _plane_field(par, st["ghost_EB"])
    gradC = np.stack([gradient(C[i], par, bc[i]) for i in range(N)])      # [N, 3, ...]
    lapC = np.stack([laplacian(C[i], par, bc[i]) for i in range(N)])      # [N, ...]
    gradEB = gradient(EB, par, beb)
    if par.mu_form == "factored":
        mut = potential.mu_tilde_factored(C, lapC, co, par.omega_stab)
    elif par.mu_form == "literal":
        mut = potential.mu_tilde_literal(C, lapC, co, par.omega_stab)
    elif par.mu_form == "no_phi":
        mut = potential.mu_tilde_literal(C, lapC, co, par.omega_stab, with_phi=False)
    else:
        raise ValueError(par.mu_form)
    if par.force_form == "conservative":
        F = gradEB.copy()
        for i in range(N):
            for j in range(N):
                if i != j:
                    F = F + co.kappa[i, j] * lapC[j] * gradC[i]
    elif par.force_form == "potential":
        mu = potential.mu_full(C, lapC, co)
        F = np.zeros_like(gradEB)
        for i in range(N):
            F = F + mu[i] * gradC[i]
    else:
        raise ValueError(par.force_form)
    F = F + par.body_force.reshape(3, 1, 1, 1)
    if par.hydro:
        mom = np.zeros((3,) + f.shape[1:])
        for k in range(lat.Q):
            for a in range(3):
                if lat.e[k, a] != 0:
                    mom[a] = mom[a] + lat.e[k, a] * f[k]
        v = mom + 0.5 * F
    else:
        v = np.zeros((3,) + f.shape[1:])
    s = s_k(lat, v)
    P = CS2 / (1.0 - lat.w[0]) * (f[1:].sum(axis=0) + s[0])
    istar = np.argmax(C, axis=0)                 # first index on ties
    tau = par.tau[istar]
    wp = 1.0 / tau
    if par.trt_magic > 0.0:
        wm = 1.0 / (0.5 + par.trt_magic / (tau - 0.5))
    else:
        wm = wp.copy()
    if par.solid is not None:
        # solid nodes hold no fluid: every node field is zero there
        for a in (EB, gradC, lapC, gradEB, mut, F, v, P, s):
            a[..., par.solid] = 0.0
    out = dict(C=C, EB=EB, gradC=gradC, lapC=lapC, gradEB=gradEB, mu_tilde=mut,
               F=F, v=v, P=P, s=s, tau=tau, omega_plus=wp, omega_minus=wm)
    if par.mobility == "c2c2":
        Phi = potential.flux_potentials(C, lapC, co, par.omega_stab)
        gradPhi = np.stack([gradient(Phi[j], par) for j in range(N)])   # [N, 3, ...]
        A = potential.alpha_c2c2(C)
        G = np.zeros_like(gradPhi)
        for i in range(N):
            for j in range(N):
                G[i] = G[i] + A[i, j] * gradPhi[j]
        out.update(Phi=Phi, alpha=A, G=G)
    return out


def mobility_source(lat, G, tau_g, m_star):
    """Source of the g-LBE in Appendix C: (1 - 1/(2 tau_g)) w_k m* e_k.G
    -> [Q, ...] for one component."""
    pre = (1.0 - 0.5 / tau_g) * m_star
    out = np.empty((lat.Q,) + G.shape[1:])
    for k in range(lat.Q):
        eG = sum(lat.e[k, a] * G[a] for a in range(3))
        out[k] = pre * lat.w[k] * eG
    return out


def f_equilibrium(lat, P, s):
    """Eq. feq with rho = 1; the rest direction takes (P/c_s^2)(w_0 - 1)."""
    feq = np.empty_like(s)
    feq[0] = P / CS2 * (lat.w[0] - 1.0) + s[0]
    for k in range(1, lat.Q):
        feq[k] = P / CS2 * lat.w[k] + s[k]
    return feq


def force_populations(lat, v, F):
    """Eq. hydroforce with grad rho = 0:
    F_k = w_k [e_k.F/c_s^2 + ((v.e_k)(F.e_k) - c_s^2 v.F)/c_s^4]."""
    vF = (v * F).sum(axis=0)
    out = np.empty((lat.Q,) + v.shape[1:])
    for k in range(lat.Q):
        eF = sum(lat.e[k, a] * F[a] for a in range(3))
        ev = sum(lat.e[k, a] * v[a] for a in range(3))
        out[k] = lat.w[k] * (eF / CS2 + (ev * eF - CS2 * vF) / (CS2 * CS2))
    return out


def g_equilibrium(lat, C, s, mut, m, form="rest"):
    """g^eq[N, Q, ...]; see the module docstring for the two forms."""
    N = C.shape[0]
    geq = np.empty((N, lat.Q) + C.shape[1:])
    for i in range(N):
        geq[i, 0] = C[i] * (1.0 + s[0]) + (1.0 - lat.w[0]) * m * mut[i]
        for k in range(1, lat.Q):
            geq[i, k] = C[i] * s[k] - lat.w[k] * m * mut[i]
        if form == "printed":
            geq[i, 0] = geq[i, 0] - C[i] + lat.w[0] * C[i]
            for k in range(1, lat.Q):
                geq[i, k] = geq[i, k] + lat.w[k] * C[i]
        elif form != "rest":
            raise ValueError(form)
    return geq


def collide(f, g, par, mac=None):
    """Steps 8-9: post-collision f*, g* (before streaming)."""
    lat = par.lat
    if mac is None:
        mac = macroscopic(f, g, par)
    s, wp, wm = mac["s"], mac["omega_plus"], mac["omega_minus"]
    if par.hydro:
        feq = f_equilibrium(lat, mac["P"], s)
        Fk = force_populations(lat, mac["v"], mac["F"])
        fs = np.empty_like(f)
        for k in range(lat.Q):
            kb = lat.opp[k]
            fp, fm = 0.5 * (f[k] + f[kb]), 0.5 * (f[k] - f[kb])
            ep, em = 0.5 * (feq[k] + feq[kb]), 0.5 * (feq[k] - feq[kb])
            fs[k] = (f[k] - wp * (fp - ep) - wm * (fm - em)
                     + 0.5 * (1.0 - 0.5 * wp) * (Fk[k] + Fk[kb])
                     + 0.5 * (1.0 - 0.5 * wm) * (Fk[k] - Fk[kb]))
    else:
        fs = f.copy()
    m_geq = 0.0 if par.mobility == "c2c2" else par.m
    geq = g_equilibrium(lat, mac["C"], s, mac["mu_tilde"], m_geq, par.geq_form)
    gs = g - (g - geq) / par.tau_g.reshape(-1, 1, 1, 1, 1)
    if par.mobility == "c2c2":
        for i in par.evolved:
            gs[i] = gs[i] + mobility_source(lat, mac["G"][i], par.tau_g[i], par.m_star)
    gs[par.implicit] = 0.0
    return fs, gs, mac


def open_face_terms(par):
    """Per open face: the f correction 2 w_k (e_k . v_b) / c_s^2 [Q] and, per
    component, g^eq_k + g^eq_kbar of (C_b, v_b) [N, Q] (rest form, mu~ of the
    uniform state C_b)."""
    lat, N = par.lat, par.N
    out = {}
    for face, (vb, Cb) in par.open_faces.items():
        v = vb.reshape(3, 1, 1, 1)
        sk = s_k(lat, v)[:, 0, 0, 0]
        mut = potential.mu_tilde_factored(Cb.reshape(N, 1), np.zeros((N, 1)), par.co,
                                          par.omega_stab)[:, 0]
        fc = np.array([lat.w[k] * (lat.e[k] @ vb) / CS2 * 2.0 for k in range(lat.Q)])
        gs = np.zeros((N, lat.Q))
        for i in range(N):
            for k in range(1, lat.Q):
                kb = lat.opp[k]
                gs[i, k] = (Cb[i] * sk[k] - lat.w[k] * par.m * mut[i]
                            + Cb[i] * sk[kb] - lat.w[kb] * par.m * mut[i])
        out[face] = (fc, gs)
    return out


def stream(post, par, kind=None):
    """Step 10 for one population array [..., Q, nz, ny, nx]; kind "f" or "g"
    selects the open-face rule."""
    lat = par.lat
    out = np.empty_like(post)
    for k in range(lat.Q):
        e = lat.e[k]
        out[..., k, :, :, :] = np.roll(post[..., k, :, :, :],
                                       shift=(int(e[2]), int(e[1]), int(e[0])),
                                       axis=(-3, -2, -1))
    # halfway bounce-back: a population leaving x towards a wall returns to x
    # reversed, which overwrites the value the periodic roll brought in.
    for k in range(1, lat.Q):
        e = lat.e[k]
        mask = wall_mask(par, e)                 # x + e_k inside a wall
        if mask.any():
            kb = lat.opp[k]
            out[..., kb, :, :, :] = np.where(mask, post[..., k, :, :, :],
                                             out[..., kb, :, :, :])
    if par.open_faces or par.outflow is not None:
        terms = open_face_terms(par)
        for k in range(1, lat.Q):
            kb = lat.opp[k]
            for face, m in open_face_masks(par, lat.e[k]).items():
                if face not in terms:
                    continue          # the outflow face: replaced after streaming
                fc, gs = terms[face]
                if kind == "f":
                    val = post[..., k, :, :, :] + fc[kb]
                elif kind == "g":
                    val = -post[..., k, :, :, :] + gs[:, kb].reshape((-1,) + (1,) * 3)
                else:
                    raise ValueError("open faces need kind='f' or 'g'")
                out[..., kb, :, :, :] = np.where(m, val, out[..., kb, :, :, :])
    if par.solid is not None:
        out[..., par.solid] = 0.0       # nothing streams into a solid node
    return out


def _plane(par, k_off=0):
    """Index tuple of the plane of the outflow face (k_off = 1: the plane
    inside it) over [..., nz, ny, nx]."""
    a = par.outflow // 2
    n = par.shape[a]
    pos = (n - 1 - k_off) if par.outflow % 2 == 1 else k_off
    idx = [slice(None)] * 3
    idx[2 - a] = pos
    return (Ellipsis,) + tuple(idx)


def _plane_field(par, plane):
    """A plane array broadcast to the lattice (its values matter only beyond
    the outflow face, where neighbour() reads them)."""
    a = par.outflow // 2
    shape = list(par.grid)
    shape[2 - a] = 1
    return np.broadcast_to(plane.reshape(shape), par.grid)


def _outflow_start(f, g, par):
    """Outflow state at t = 0: the boundary plane's populations, U = 0 and
    ghosts equal to the boundary plane's C and E_B."""
    if par.outflow is None:
        return
    C = concentrations(g, par)
    EB = potential.bulk_energy(C, par.co)
    bn = _plane(par)
    par.outflow_state = {"f": f[bn].copy(), "g": g[bn].copy(), "U": 0.0,
                         "ghost_C": C[bn].copy(), "ghost_EB": EB[bn].copy()}


def _outflow_apply(f, g, par):
    """Eq. convect on the streamed populations, then the ghosts."""
    st = par.outflow_state
    a = par.outflow // 2
    sgn = 1.0 if par.outflow % 2 == 1 else -1.0
    lat = par.lat
    inner = _plane(par, 1)
    mom = np.zeros(f[0][inner[1:]].shape)
    for k in range(1, lat.Q):
        if lat.e[k, a] != 0:
            mom = mom + sgn * lat.e[k, a] * f[k][inner[1:]]
    # the mean over the fluid nodes of plane N-1 (solid nodes hold no fluid)
    fluid = np.ones(mom.shape, dtype=bool) if par.solid is None else ~par.solid[inner[1:]]
    U = max(float(mom[fluid].mean()), 0.0)
    bn = _plane(par)
    f[bn] = (st["f"] + U * f[inner]) / (1.0 + U)
    g[bn] = (st["g"] + U * g[inner]) / (1.0 + U)
    g[par.implicit] = 0.0
    st["f"], st["g"], st["U"] = f[bn].copy(), g[bn].copy(), U
    C = concentrations(g, par)
    EB = potential.bulk_energy(C, par.co)
    st["ghost_C"] = (st["ghost_C"] + U * C[bn]) / (1.0 + U)
    st["ghost_EB"] = (st["ghost_EB"] + U * EB[bn]) / (1.0 + U)


def step(f, g, par):
    """One full time step; returns (f, g, mac) with mac the macroscopic fields
    of the input state."""
    fs, gs, mac = collide(f, g, par)
    gn = stream(gs, par, "g")
    gn[par.implicit] = 0.0
    fn = stream(fs, par, "f")
    if par.outflow is not None:
        _outflow_apply(fn, gn, par)
    return fn, gn, mac


def run(f, g, par, steps):
    for _ in range(steps):
        f, g, _ = step(f, g, par)
    return f, g


def initial_state(par, C0, v0=None, P0=None):
    """f = f^eq(P0, v0) and g_{i,0} = C_i, g_{i,k>=1} = 0 (initialisation is not
    specified in the paper; these values are exactly representable and are
    forgotten after one step when tau_g = 1)."""
    lat = par.lat
    C0 = np.asarray(C0, dtype=np.float64).reshape((par.N,) + par.grid)
    if v0 is None:
        v0 = np.zeros((3,) + par.grid)
    else:
        v0 = np.asarray(v0, dtype=np.float64).reshape((3,) + par.grid)
    if P0 is None:
        P0 = np.zeros(par.grid)
    else:
        P0 = np.asarray(P0, dtype=np.float64).reshape(par.grid)
    f = f_equilibrium(lat, P0, s_k(lat, v0))
    g = np.zeros((par.N, lat.Q) + par.grid)
    g[:, 0] = C0
    g[par.implicit] = 0.0
    if par.solid is not None:
        f[..., par.solid] = 0.0
        g[..., par.solid] = 0.0
    _outflow_start(f, g, par)
    return f, g
