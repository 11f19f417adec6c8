"""The time step of step.py written node by node in pure Python (FP64).

Test infrastructure only, for tiny lattices (a few hundred nodes).  It is an
independent transcription of the same definitions: explicit index arithmetic
for neighbours, walls, solid nodes and open faces (Sec. III C) instead of
array rolls and masks, and the flux
potential in the literal form of Eq. MU (sum_j alpha_ij (mu_j + phi_j + xi_j))
instead of the factored form.  Agreement with step.py therefore checks the
vectorisation and the factored algebra together (to rounding, not bitwise).
"""
import itertools
import math

import numpy as np

CS2 = 1.0 / 3.0


def _fp(c):
    return c * c * (1 - c) * (1 - c)


def _dfp(c):
    return 2 * c * (1 - 3 * c + 2 * c * c)


def _is_solid(par, x, y, z):
    return par.solid is not None and bool(par.solid[z, y, x])


def _link(par, x, y, z, e):
    """Where the link from x along e leads: (X, Y, Z) of a fluid node, None
    for a wall (a wall face or a solid node), or the open face (an int) it
    leaves across.  A link that crosses a wall face is a wall link even if
    it also crosses an open face; across two open faces it takes the first
    axis's; across an open face it is still a wall link if, with its
    component normal to the face removed, it leads to a solid node."""
    nx, ny, nz = par.shape
    n = (nx, ny, nz)
    c = (x, y, z)
    p = [c[a] + int(e[a]) for a in range(3)]
    open_face = None
    for a in range(3):
        if p[a] < 0 or p[a] >= n[a]:
            if not par.walls[a]:
                p[a] %= n[a]
                continue
            face = 2 * a + (1 if p[a] >= n[a] else 0)
            if face in par.open_faces or face == par.outflow:
                if open_face is None:
                    open_face = face
            else:
                return None
    if open_face is not None:
        t = list(p)
        t[open_face // 2] = c[open_face // 2]
        if t != list(c) and _is_solid(par, t[0], t[1], t[2]):
            return None
        return open_face
    if _is_solid(par, p[0], p[1], p[2]):
        return None
    return p[0], p[1], p[2]


def _face_values(par, face):
    """C_b, E_B(C_b), mu~(C_b) (literal form, no gradients) and v_b of an
    open face."""
    co, N = par.co, par.N
    vb, Cb = par.open_faces[face]
    eb = 0.0
    for i in range(N):
        for j in range(N):
            if i != j:
                eb += 0.5 * co.beta[i, j] * (_fp(Cb[i]) + _fp(Cb[j]) - _fp(Cb[i] + Cb[j]))
    mu = [sum(co.beta[j, k2] * (_dfp(Cb[j]) - _dfp(Cb[j] + Cb[k2])) for k2 in range(N) if k2 != j)
          for j in range(N)]
    ph = [0.0] * N
    for j in range(N):
        for k2, l, m in itertools.combinations(range(N), 3):
            if j not in (k2, l, m):
                ph[j] += 12.0 / co.D * co.Lam[j, k2, l, m] * Cb[k2] * Cb[l] * Cb[m]
    xs = [0.0] * N
    if par.omega_stab != 0.0:
        for j in range(N):
            for k2, l in itertools.combinations(range(N), 2):
                if j in (k2, l):
                    continue
                inner = 2.0 * Cb[j]
                for m in range(N):
                    if m not in (j, k2, l):
                        inner -= co.Theta[k2, l, j, m] * Cb[m]
                xs[j] += 12.0 / co.D * par.omega_stab * Cb[k2] ** 2 * Cb[l] ** 2 * inner
    mut = [sum(co.alpha[i, j] * (mu[j] + ph[j] + xs[j]) for j in range(N)) for i in range(N)]
    return list(Cb), eb, mut, list(vb)


def step(f, g, par):
    if par.outflow is not None:
        raise ValueError("the node loop has no convective outflow")
    lat, co, N = par.lat, par.co, par.N
    Q = lat.Q
    nx, ny, nz = par.shape
    D = co.D
    faces = {face: _face_values(par, face) for face in par.open_faces}
    C = np.zeros((N, nz, ny, nx))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                others = 0.0
                for i in range(N):
                    if i == par.implicit:
                        continue
                    s = 0.0
                    for k in range(Q):
                        s += g[i, k, z, y, x]
                    C[i, z, y, x] = s
                    others += s
                C[par.implicit, z, y, x] = 1.0 - others
                if _is_solid(par, x, y, z):
                    C[:, z, y, x] = 0.0
    EB = np.zeros((nz, ny, nx))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                s = 0.0
                for i in range(N):
                    for j in range(N):
                        if i != j:
                            ci, cj = C[i, z, y, x], C[j, z, y, x]
                            s += 0.5 * co.beta[i, j] * (_fp(ci) + _fp(cj) - _fp(ci + cj))
                EB[z, y, x] = s
    fnew = np.zeros_like(f)
    gnew = np.zeros_like(g)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if _is_solid(par, x, y, z):
                    continue              # no fluid, nothing collides or streams
                nb = [_link(par, x, y, z, lat.e[k]) for k in range(Q)]
                c0 = [C[i, z, y, x] for i in range(N)]
                grad = [[0.0, 0.0, 0.0] for _ in range(N)]
                lap = [0.0] * N
                gE = [0.0, 0.0, 0.0]
                for k in range(1, Q):
                    if nb[k] is None:
                        continue          # neighbour in the wall: psi(x) - psi(x) = 0
                    if isinstance(nb[k], int):
                        # beyond an open face: the face's boundary values
                        cn, en = faces[nb[k]][0], faces[nb[k]][1]
                    else:
                        X, Y, Z = nb[k]
                        cn = [C[i, Z, Y, X] for i in range(N)]
                        en = EB[Z, Y, X]
                    for i in range(N):
                        d = cn[i] - c0[i]
                        lap[i] += 2.0 / CS2 * lat.w[k] * d
                        for a in range(3):
                            grad[i][a] += lat.w[k] * lat.e[k, a] * d / CS2
                    dE = en - EB[z, y, x]
                    for a in range(3):
                        gE[a] += lat.w[k] * lat.e[k, a] * dE / CS2
                # chemical potentials (Eq. mu), phi (Eq. G), xi (Eq. P)
                mu = [0.0] * N
                for j in range(N):
                    for k2 in range(N):
                        if k2 != j:
                            mu[j] += (co.beta[j, k2] * (_dfp(c0[j]) - _dfp(c0[j] + c0[k2]))
                                      + co.kappa[j, k2] * lap[k2])
                ph = [0.0] * N
                for j in range(N):
                    for k2, l, m in itertools.combinations(range(N), 3):
                        if j not in (k2, l, m):
                            ph[j] += 12.0 / D * co.Lam[j, k2, l, m] * c0[k2] * c0[l] * c0[m]
                xs = [0.0] * N
                if par.omega_stab != 0.0:
                    for j in range(N):
                        for k2, l in itertools.combinations(range(N), 2):
                            if j in (k2, l):
                                continue
                            inner = 2.0 * c0[j]
                            for m in range(N):
                                if m not in (j, k2, l):
                                    inner -= co.Theta[k2, l, j, m] * c0[m]
                            xs[j] += 12.0 / D * par.omega_stab * c0[k2] ** 2 * c0[l] ** 2 * inner
                mut = [sum(co.alpha[i, j] * (mu[j] + ph[j] + xs[j]) for j in range(N))
                       for i in range(N)]
                if par.force_form == "conservative":
                    F = list(gE)
                    for i in range(N):
                        for j in range(N):
                            if i != j:
                                for a in range(3):
                                    F[a] += co.kappa[i, j] * lap[j] * grad[i][a]
                else:
                    F = [0.0, 0.0, 0.0]
                    for i in range(N):
                        for a in range(3):
                            F[a] += mu[i] * grad[i][a]
                for a in range(3):
                    F[a] += par.body_force[a]
                fl = [f[k, z, y, x] for k in range(Q)]
                v = [0.0, 0.0, 0.0]
                if par.hydro:
                    for a in range(3):
                        v[a] = sum(lat.e[k, a] * fl[k] for k in range(Q)) + 0.5 * F[a]
                vv = v[0] ** 2 + v[1] ** 2 + v[2] ** 2
                sk = []
                for k in range(Q):
                    ev = lat.e[k, 0] * v[0] + lat.e[k, 1] * v[1] + lat.e[k, 2] * v[2]
                    sk.append(lat.w[k] * (3 * ev + 4.5 * ev * ev - 1.5 * vv))
                P = CS2 / (1 - lat.w[0]) * (sum(fl[1:]) + sk[0])
                best = 0
                for i in range(1, N):
                    if c0[i] > c0[best]:
                        best = i
                tau = par.tau[best]
                wp = 1.0 / tau
                wm = wp if par.trt_magic <= 0 else 1.0 / (0.5 + par.trt_magic / (tau - 0.5))
                feq = [P / CS2 * (lat.w[0] - 1) + sk[0]] + [P / CS2 * lat.w[k] + sk[k]
                                                             for k in range(1, Q)]
                vF = v[0] * F[0] + v[1] * F[1] + v[2] * F[2]
                Fk = []
                for k in range(Q):
                    eF = lat.e[k, 0] * F[0] + lat.e[k, 1] * F[1] + lat.e[k, 2] * F[2]
                    ev = lat.e[k, 0] * v[0] + lat.e[k, 1] * v[1] + lat.e[k, 2] * v[2]
                    Fk.append(lat.w[k] * (3 * eF + 9 * ev * eF - 3 * vF))
                for k in range(Q):
                    kb = lat.opp[k]
                    if par.hydro:
                        post = (fl[k] - wp * ((fl[k] + fl[kb]) / 2 - (feq[k] + feq[kb]) / 2)
                                - wm * ((fl[k] - fl[kb]) / 2 - (feq[k] - feq[kb]) / 2)
                                + 0.5 * (1 - 0.5 * wp) * (Fk[k] + Fk[kb])
                                + 0.5 * (1 - 0.5 * wm) * (Fk[k] - Fk[kb]))
                    else:
                        post = fl[k]
                    dst = nb[k]
                    if dst is None:
                        fnew[kb, z, y, x] = post
                    elif isinstance(dst, int):
                        # velocity Dirichlet: back along kb with 2 w_kb (e_kb . v_b) / c_s^2
                        vb = faces[dst][3]
                        ekv = sum(lat.e[kb, a] * vb[a] for a in range(3))
                        fnew[kb, z, y, x] = post + 2.0 * lat.w[kb] * ekv / CS2
                    else:
                        fnew[k, dst[2], dst[1], dst[0]] = post
                for i in range(N):
                    if i == par.implicit:
                        continue
                    for k in range(Q):
                        if k == 0:
                            geq = c0[i] * (1 + sk[0]) + (1 - lat.w[0]) * par.m * mut[i]
                        else:
                            geq = c0[i] * sk[k] - lat.w[k] * par.m * mut[i]
                        post = g[i, k, z, y, x] - (g[i, k, z, y, x] - geq) / par.tau_g[i]
                        dst = nb[k]
                        if dst is None:
                            gnew[i, lat.opp[k], z, y, x] = post
                        elif isinstance(dst, int):
                            # anti-bounce-back: minus it plus g^eq_k + g^eq_kb of the face
                            Cb, _, mub, vb = faces[dst]
                            vvb = vb[0] ** 2 + vb[1] ** 2 + vb[2] ** 2
                            eq = 0.0
                            for q in (k, lat.opp[k]):
                                ev = lat.e[q, 0] * vb[0] + lat.e[q, 1] * vb[1] + lat.e[q, 2] * vb[2]
                                sq = lat.w[q] * (3 * ev + 4.5 * ev * ev - 1.5 * vvb)
                                eq += Cb[i] * sq - lat.w[q] * par.m * mub[i]
                            gnew[i, lat.opp[k], z, y, x] = -post + eq
                        else:
                            gnew[i, k, dst[2], dst[1], dst[0]] = post
    return fnew, gnew


def total(values):
    return math.fsum(float(v) for v in np.ravel(values))
