"""Closed forms and measurements used as pins (FP64).  Test infrastructure only.

* neumann_angle: Eq. neucosine, cos(pi - theta_ij) = -(s_ij^2 - s_ik^2 - s_jk^2)
  / (2 s_ik s_jk).  theta_ij is the angle filled by the third fluid k.
* layered_poiseuille: Eqs. piecewisequad and velocityprof.  Per layer n,
  v_n(x) = sgn F/(2 eta_n) x^2 + A/eta_n x + B_n, with v_1(0) = 0, v_L(W) = 0 and
  v continuous at each interface (continuous shear stress gives one constant A).
  The paper writes eta v'' = +F (sgn = +1), which with its printed A < 0 is the
  profile of a force pointing against +v; the physical balance of a body force
  driving the flow is eta v'' = -F (sgn = -1).
* linear_growth: the linear response of the Cahn-Hilliard LBE with tau_g = 1 and
  v = 0.  Streaming the rest-form equilibrium gives
  C(t+1) = C(t) - (m/6) lap mu~, and linearising mu~ = a dC + (3D/4) lap dC gives
  per Fourier mode G(k) = 1 + M lam(k) (a - (3D/4) lam(k)), with M = m/6 and
  lam(k) = (2/c_s^2) sum_q w_q (1 - cos k.e_q) the symbol of -lap.
* lens_angles: fit circles to the upper and lower C = 1/2 contour of a lens and
  take the angles between the circles and the flat interface at the triple
  points (the measurement described after Eq. neucosine).
"""
import math

import numpy as np


def neumann_angle(s_ij, s_ik, s_jk):
    """theta_ij in degrees (Eq. neucosine)."""
    c = -(s_ij ** 2 - s_ik ** 2 - s_jk ** 2) / (2.0 * s_ik * s_jk)
    return 180.0 - math.degrees(math.acos(c))


def layered_poiseuille(edges, eta, F, sign=-1.0):
    """Constants (A, B[0..L-1]) of the layered profile.

    edges: [0, x_1, ..., x_{L-1}, W] layer boundaries (walls at 0 and W);
    eta: L viscosities; F: body force; sign: -1 physical, +1 as printed.
    """
    L = len(eta)
    edges = np.asarray(edges, dtype=np.float64)
    assert len(edges) == L + 1
    n = L + 1                     # unknowns A, B_1..B_L
    M = np.zeros((n, n))
    b = np.zeros(n)

    def row_v(layer, x):
        r = np.zeros(n)
        r[0] = x / eta[layer]
        r[1 + layer] = 1.0
        return r, sign * F / (2.0 * eta[layer]) * x * x

    r, c = row_v(0, edges[0])
    M[0], b[0] = r, -c
    for q in range(1, L):
        r1, c1 = row_v(q - 1, edges[q])
        r2, c2 = row_v(q, edges[q])
        M[q], b[q] = r1 - r2, -(c1 - c2)
    r, c = row_v(L - 1, edges[L])
    M[L], b[L] = r, -c
    x = np.linalg.solve(M, b)
    return x[0], x[1:]


def layered_profile(x, edges, eta, F, sign=-1.0):
    A, B = layered_poiseuille(edges, eta, F, sign)
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for q in range(len(eta)):
        sel = (x >= edges[q]) & (x <= edges[q + 1])
        out[sel] = sign * F / (2 * eta[q]) * x[sel] ** 2 + A / eta[q] * x[sel] + B[q]
    return out


def laplacian_symbol(lat, kvec):
    """lam(k) = (2/c_s^2) sum_{q>=1} w_q (1 - cos(k . e_q)) for k [3, ...]."""
    out = 0.0
    for q in range(1, lat.Q):
        ke = sum(kvec[a] * lat.e[q, a] for a in range(3))
        out = out + lat.w[q] * (1.0 - np.cos(ke))
    return 6.0 * out


def linear_growth(lam, M, a, D):
    return 1.0 + M * lam * (a - 0.75 * D * lam)


def gradient_symbol(lat, kvec):
    """s(k) = sum_{q>=1} w_q e_q sin(k . e_q) -> [3]: the isotropic gradient
    (1/c_s^2) sum_q w_q e_q [psi(x + e_q) - psi(x)] acts on exp(i k.x) as
    3 i s(k)."""
    out = np.zeros(3)
    for q in range(1, lat.Q):
        ke = sum(kvec[a] * lat.e[q, a] for a in range(3))
        out = out + lat.w[q] * lat.e[q] * np.sin(ke)
    return out


def source_mobility_growth(lat, kvec, alpha0, A, kappa, m_star, tau_g=1.0):
    """Per-step growth matrix of a Fourier mode of C about a uniform state in
    the concentration-dependent mobility scheme of Appendix C, tau_g = 1,
    v = 0.  With g^eq carrying no mobility term, C(x, t+1) = C(x, t) +
    sum_k S_k(x - e_k) for the source S_k = (1/2) w_k m* e_k.G, and G =
    alpha0 grad Phi; streaming turns the sum into (3/2) m* |s(k)|^2 times G's
    amplitude over 3 i s(k).  Phi linearises as (A - K lam(k)) dC with A the
    Jacobian of the bulk part of mu + phi + xi and K_jk = kappa_jk (j != k)
    from the gradient part of mu_j.  Returns the N x N matrix."""
    if tau_g != 1.0:
        raise ValueError("closed form holds for tau_g = 1")
    s = gradient_symbol(lat, kvec)
    lam = laplacian_symbol(lat, kvec)
    K = np.array(kappa, dtype=np.float64).copy()
    np.fill_diagonal(K, 0.0)
    N = K.shape[0]
    return np.eye(N) + 1.5 * m_star * float(s @ s) * (alpha0 @ (A - K * lam))


def laplace_pressure_2d(sigma, R):
    return sigma / R


def laplace_pressure_3d(sigma, R):
    return 2.0 * sigma / R


def _fit_circle(px, py):
    """Algebraic least-squares circle: x^2 + y^2 + a x + b y + c = 0."""
    A = np.stack([px, py, np.ones_like(px)], axis=1)
    rhs = -(px ** 2 + py ** 2)
    (a, b, c), *_ = np.linalg.lstsq(A, rhs, rcond=None)
    xc, yc = -a / 2, -b / 2
    return xc, yc, math.sqrt(xc * xc + yc * yc - c)


def contour_points(field, level=0.5):
    """Sub-node crossings of ``field`` = level along x and y grid lines of a 2-D
    array [ny, nx] (linear interpolation, no wrap)."""
    ny, nx = field.shape
    pts = []
    for j in range(ny):
        row = field[j]
        for i in range(nx - 1):
            a, b = row[i] - level, row[i + 1] - level
            if a == 0.0 or a * b < 0:
                pts.append((i + a / (a - b), j))
    for i in range(nx):
        col = field[:, i]
        for j in range(ny - 1):
            a, b = col[j] - level, col[j + 1] - level
            if a == 0.0 or a * b < 0:
                pts.append((i, j + a / (a - b)))
    return np.array(pts, dtype=np.float64).reshape(-1, 2)


def lens_angles(C_lens, y_interface, margin=3.0):
    """Angles of a lens of one fluid sitting on a flat horizontal interface.

    C_lens: [ny, nx] concentration of the lens fluid; y_interface: the height
    of the flat interface.  Contour points above (below) y_interface + margin
    (- margin) are fitted with one circle each.  Returns a dict of the lens
    angle (filled by the lens fluid) and the angles filled by the fluids above
    and below, in degrees, averaged over the two triple points.
    """
    pts = contour_points(C_lens)
    top = pts[pts[:, 1] > y_interface + margin]
    bot = pts[pts[:, 1] < y_interface - margin]
    xt, yt, rt = _fit_circle(top[:, 0], top[:, 1])
    xb, yb, rb = _fit_circle(bot[:, 0], bot[:, 1])
    res = {"top_circle": (xt, yt, rt), "bottom_circle": (xb, yb, rb)}

    def cap_angle(xc, yc, r, above):
        # half-chord where the circle crosses the interface line
        dy = y_interface - yc
        half = math.sqrt(max(r * r - dy * dy, 0.0))
        # angle between the tangent at the crossing and the interface line
        # equals the angle between the radius there and the vertical.
        ang = math.degrees(math.acos(max(-1.0, min(1.0, abs(dy) / r))))
        centre_on_far_side = (yc < y_interface) if above else (yc > y_interface)
        return (ang if centre_on_far_side else 180.0 - ang), half

    a_top, _ = cap_angle(xt, yt, rt, True)
    a_bot, _ = cap_angle(xb, yb, rb, False)
    res["psi_top"] = a_top
    res["psi_bottom"] = a_bot
    res["lens"] = a_top + a_bot
    res["above"] = 180.0 - a_top
    res["below"] = 180.0 - a_bot
    return res


def janus_lens_angles(C_a, C_b, y_interface, x_split, margin=3.0):
    """Angles at the outer triple points of a Janus lens: fluids a (left of
    x = x_split) and b (right) together form a lens on a flat horizontal
    interface between an upper and a lower fluid (Sec. IV A, Table I).

    For each lens fluid, the part of its C = 0.5 contour away from the a|b
    interface (|x - x_split| > margin) and from the flat interface
    (|y - y_interface| > margin) is fitted with one circle above and one below
    the interface, as in lens_angles; the interior angle is the one filled by
    the lens fluid at its outer triple point.  Returns the interior angle and
    the angles filled by the upper and lower fluids, averaged over a and b,
    plus the per-fluid values."""
    res = {}
    for name, C, side in (("a", C_a, -1.0), ("b", C_b, 1.0)):
        pts = contour_points(C)
        pts = pts[side * (pts[:, 0] - x_split) > margin]
        top = pts[pts[:, 1] > y_interface + margin]
        bot = pts[pts[:, 1] < y_interface - margin]
        xt, yt, rt = _fit_circle(top[:, 0], top[:, 1])
        xb, yb, rb = _fit_circle(bot[:, 0], bot[:, 1])
        a_top = _cap_angle(yt, rt, y_interface, True)
        a_bot = _cap_angle(yb, rb, y_interface, False)
        res[name] = {"interior": a_top + a_bot, "above": 180.0 - a_top, "below": 180.0 - a_bot}
    for key in ("interior", "above", "below"):
        res[key] = 0.5 * (res["a"][key] + res["b"][key])
    return res


def _cap_angle(yc, r, y_interface, above):
    """Angle between a circular arc and the horizontal line y = y_interface at
    their crossing, measured inside the cap on the given side of the line."""
    dy = y_interface - yc
    ang = math.degrees(math.acos(max(-1.0, min(1.0, abs(dy) / r))))
    centre_on_far_side = (yc < y_interface) if above else (yc > y_interface)
    return ang if centre_on_far_side else 180.0 - ang


def domain_size(C, level=0.5):
    """Characteristic length L_i of each component (Eq. L, Sec. IV B).

    C: [N, nz, ny, nx] (or [N, ny, nx]).  lambda_i = H(C_i - level), taken as
    C_i > level; S_i(k) = |sum_x lambda_i(x) exp(-i k.x)|^2 on the periodic
    lattice's wave vectors k = 2 pi (m_x/nx, m_y/ny, m_z/nz).  The integrals
    of Eq. L become sums over the full k grid (circular averaging followed by
    integration over d^2k visits every k once); k = 0, which carries only the
    mean of lambda, is left out of both.  L_i = 2 pi sum S_i / sum |k| S_i."""
    C = np.asarray(C, dtype=np.float64)
    if C.ndim == 3:
        C = C[:, None]
    N = C.shape[0]
    shape = C.shape[1:]
    freqs = [2.0 * np.pi * np.fft.fftfreq(n) for n in shape]
    kz, ky, kx = np.meshgrid(*freqs, indexing="ij")
    kmag = np.sqrt(kx * kx + ky * ky + kz * kz)
    nonzero = kmag > 0
    out = np.empty(N)
    for i in range(N):
        lam = (C[i] > level).astype(np.float64)
        S = np.abs(np.fft.fftn(lam)) ** 2
        out[i] = 2.0 * np.pi * S[nonzero].sum() / (kmag[nonzero] * S[nonzero]).sum()
    return out
