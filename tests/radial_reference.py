"""1-D references for the spherical shock-tube problems (test infrastructure).

* ``exact_sod`` — the exact solution of the planar Riemann problem for the
  Euler equations (two-shock/rarefaction wave curves, Newton iteration on the
  star pressure), sampled at x / t.
* ``spherical_euler`` — a fine-grid finite-volume solution of the
  spherically symmetric Euler equations
      d(r^2 U)/dt + d(r^2 F)/dr = (0, 2 r p, 0)
  (second order: MUSCL with minmod-limited primitive slopes, HLL fluxes,
  Heun's method in time, zero-gradient ends).  With ``planar=True`` the
  r^2 weights and the source are dropped, which turns it into the planar
  scheme that the exact solution pins.
* ``mhd_equator`` — the same kind of scheme for ideal MHD in the equatorial
  plane of a spherical problem with no theta or phi dependence: variables
  (rho, rho v_r, rho v_phi, E, B_phi) with the radial field B_r = C / r^2
  fixed, each conserved in its own radial weight,
      d(r^m q)/dt + d(r^m F)/dr = r^m S,  m = (2, 2, 3, 2, 1),
  and the one source S_r = (2 p + B_r^2 + rho v_phi^2) / r of the radial
  momentum (the B_phi pressure and hoop stress cancel); the B_r^2 part of the
  source is integrated exactly over each cell, so a uniform state threaded by
  B_r = C / r^2 stays at rest.  HLL with fast-magnetosonic Davis speeds.
  With ``planar=True`` the weights and the source are dropped and B_r = C.

Neither shares anything with the library or the oracle; they give the
physical solution the 3-D step must approach on a spherically symmetric
problem.
"""
import numpy as np


def _sound(p, rho, gam):
    return np.sqrt(gam * p / rho)


def exact_sod(xi, rhoL, pL, uL, rhoR, pR, uR, gam):
    """Exact planar Riemann solution at similarity coordinates xi = (x - x0)/t."""
    cL, cR = _sound(pL, rhoL, gam), _sound(pR, rhoR, gam)

    def f(p, rho, pk, ck):
        if p > pk:   # shock
            A, B = 2.0 / ((gam + 1) * rho), (gam - 1) / (gam + 1) * pk
            return (p - pk) * np.sqrt(A / (p + B)), np.sqrt(A / (p + B)) * (1 - 0.5 * (p - pk) / (p + B))
        r = (p / pk) ** ((gam - 1) / (2 * gam))   # rarefaction
        return 2 * ck / (gam - 1) * (r - 1), 1.0 / (rho * ck) * (p / pk) ** (-(gam + 1) / (2 * gam))

    p = 0.5 * (pL + pR)
    for _ in range(100):
        fl, dl = f(p, rhoL, pL, cL)
        fr, dr = f(p, rhoR, pR, cR)
        dp = (fl + fr + uR - uL) / (dl + dr)
        p = max(p - dp, 1e-12)
        if abs(dp) < 1e-14 * p:
            break
    fl, _ = f(p, rhoL, pL, cL)
    fr, _ = f(p, rhoR, pR, cR)
    us = 0.5 * (uL + uR) + 0.5 * (fr - fl)
    out = np.zeros((3, len(xi)))
    g1, g2 = (gam - 1) / (gam + 1), (gam - 1) / (2 * gam)
    for n, s in enumerate(xi):
        if s <= us:   # left of the contact
            if p > pL:
                rs = rhoL * (p / pL + g1) / (g1 * p / pL + 1)
                S = uL - cL * np.sqrt((gam + 1) / (2 * gam) * p / pL + g2)
                out[:, n] = (rhoL, uL, pL) if s < S else (rs, us, p)
            else:
                cs = cL * (p / pL) ** g2
                if s < uL - cL:
                    out[:, n] = (rhoL, uL, pL)
                elif s > us - cs:
                    out[:, n] = (rhoL * (p / pL) ** (1 / gam), us, p)
                else:
                    u = 2 / (gam + 1) * (cL + (gam - 1) / 2 * uL + s)
                    c = 2 / (gam + 1) * (cL + (gam - 1) / 2 * (uL - s))
                    rho = rhoL * (c / cL) ** (2 / (gam - 1))
                    out[:, n] = (rho, u, pL * (c / cL) ** (2 * gam / (gam - 1)))
        else:
            if p > pR:
                rs = rhoR * (p / pR + g1) / (g1 * p / pR + 1)
                S = uR + cR * np.sqrt((gam + 1) / (2 * gam) * p / pR + g2)
                out[:, n] = (rhoR, uR, pR) if s > S else (rs, us, p)
            else:
                cs = cR * (p / pR) ** g2
                if s > uR + cR:
                    out[:, n] = (rhoR, uR, pR)
                elif s < us + cs:
                    out[:, n] = (rhoR * (p / pR) ** (1 / gam), us, p)
                else:
                    u = 2 / (gam + 1) * (-cR + (gam - 1) / 2 * uR + s)
                    c = 2 / (gam + 1) * (cR - (gam - 1) / 2 * (uR - s))
                    rho = rhoR * (c / cR) ** (2 / (gam - 1))
                    out[:, n] = (rho, u, pR * (c / cR) ** (2 * gam / (gam - 1)))
    return out   # rho, u, p


def _minmod(a, b):
    return np.where(a * b > 0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


def spherical_euler(r_in, r_out, n, r0, left, right, gam, t_end, cfl=0.4, planar=False):
    """Cell-centred radii and (rho, u, p) at t_end for a jump at r0 between the
    primitive states left = (rho, u, p) and right."""
    edges = np.linspace(r_in, r_out, n + 1)
    rc = 0.5 * (edges[:-1] + edges[1:])
    dr = edges[1] - edges[0]
    if planar:
        wf = np.ones(n + 1)
        vol = np.full(n, dr)
    else:
        wf = edges ** 2
        vol = (edges[1:] ** 3 - edges[:-1] ** 3) / 3.0
    W = np.where(rc <= r0, 1.0, 0.0)
    rho = W * left[0] + (1 - W) * right[0]
    u = W * left[1] + (1 - W) * right[1]
    p = W * left[2] + (1 - W) * right[2]
    U = np.array([rho, rho * u, p / (gam - 1) + 0.5 * rho * u * u])

    def prim(U):
        rho = U[0]
        u = U[1] / rho
        return rho, u, (gam - 1) * (U[2] - 0.5 * rho * u * u)

    def rhs(U):
        rho, u, p = prim(U)
        q = np.array([rho, u, p])
        qg = np.concatenate([q[:, :1], q[:, :1], q, q[:, -1:], q[:, -1:]], axis=1)
        d = _minmod(qg[:, 1:-1] - qg[:, :-2], qg[:, 2:] - qg[:, 1:-1])   # slopes of cells -1 .. n
        qL = qg[:, 1:-2] + 0.5 * d[:, :-1]    # left state at faces 0 .. n
        qR = qg[:, 2:-1] - 0.5 * d[:, 1:]     # right state at faces 0 .. n

        def cons(q):
            return np.array([q[0], q[0] * q[1], q[2] / (gam - 1) + 0.5 * q[0] * q[1] ** 2])

        def flux(q):
            return np.array([q[0] * q[1], q[0] * q[1] ** 2 + q[2],
                             q[1] * (q[2] / (gam - 1) + 0.5 * q[0] * q[1] ** 2 + q[2])])

        cL, cR = _sound(qL[2], qL[0], gam), _sound(qR[2], qR[0], gam)
        sL = np.minimum(qL[1] - cL, qR[1] - cR)
        sR = np.maximum(qL[1] + cL, qR[1] + cR)
        FL, FR, UL, UR = flux(qL), flux(qR), cons(qL), cons(qR)
        Fh = np.where(sL >= 0, FL, np.where(sR <= 0, FR, (sR * FL - sL * FR + sL * sR * (UR - UL)) / (sR - sL)))
        Fw = Fh * wf
        out = -(Fw[:, 1:] - Fw[:, :-1]) / vol
        if not planar:
            out[1] += p * (edges[1:] ** 2 - edges[:-1] ** 2) / vol   # 2 r p, integrated over the cell
        return out

    t = 0.0
    while t < t_end:
        rho, u, p = prim(U)
        dt = cfl * dr / np.max(np.abs(u) + _sound(p, rho, gam))
        dt = min(dt, t_end - t)
        U1 = U + dt * rhs(U)
        U = 0.5 * (U + U1 + dt * rhs(U1))
        t += dt
    return rc, np.array(prim(U))


def _fast(rho, p, bn, bt, gam):
    a2, n2, t2 = gam * p / rho, bn * bn / rho, bt * bt / rho
    s = a2 + n2 + t2
    return np.sqrt(0.5 * (s + np.sqrt(np.maximum(s * s - 4.0 * a2 * n2, 0.0))))


def mhd_equator(r_in, r_out, n, rm, left, right, C, gam, t_end, cfl=0.4, planar=False, init=None):
    """Cell-centred radii and (rho, v_r, v_phi, p, B_phi) at t_end.  left and
    right are (rho, p, v_r, v_phi, B_phi) inside and outside r = rm; init, if
    given, maps the cell centres to those five primitive arrays instead."""
    edges = np.linspace(r_in, r_out, n + 1)
    rc = 0.5 * (edges[:-1] + edges[1:])
    dr = edges[1] - edges[0]
    m = np.array([0, 0, 0, 0, 0]) if planar else np.array([2, 2, 3, 2, 1])
    wf = edges[None, :] ** m[:, None]                                     # face weights r^m
    vol = (edges[None, 1:] ** (m[:, None] + 1) - edges[None, :-1] ** (m[:, None] + 1)) / (m[:, None] + 1)
    if planar:
        Brf = np.full(n + 1, C)
        Br2c = np.full(n, C * C)
    else:
        Brf = C / edges ** 2
        Br2c = C * C * (1.0 / edges[:-1] - 1.0 / edges[1:]) / vol[0]      # cell average of B_r^2 (weight r^2)
    if init is None:
        inner = rc <= rm
        w0 = [np.where(inner, a, b) for a, b in zip(left, right)]
        rho, p, vr, vp, bp = w0
    else:
        rho, p, vr, vp, bp = init(rc)

    def cons(rho, vr, vp, p, bp, br2):
        return np.array([rho, rho * vr, rho * vp, p / (gam - 1) + 0.5 * rho * (vr * vr + vp * vp) + 0.5 * (br2 + bp * bp), bp])

    def prim(U):
        rho = U[0]
        vr, vp = U[1] / rho, U[2] / rho
        p = (gam - 1) * (U[3] - 0.5 * rho * (vr * vr + vp * vp) - 0.5 * (Br2c + U[4] ** 2))
        return rho, vr, vp, p, U[4]

    def flux(rho, vr, vp, p, bp, br):
        ps = p + 0.5 * (br * br + bp * bp)
        E = p / (gam - 1) + 0.5 * rho * (vr * vr + vp * vp) + 0.5 * (br * br + bp * bp)
        return np.array([rho * vr, rho * vr * vr + ps - br * br, rho * vr * vp - br * bp,
                         (E + ps) * vr - br * (vr * br + vp * bp), vr * bp - vp * br])

    U = cons(rho, vr, vp, p, bp, Br2c)

    def rhs(U):
        q = np.array(prim(U))                                 # rho, vr, vp, p, bp
        qg = np.concatenate([q[:, :1], q[:, :1], q, q[:, -1:], q[:, -1:]], axis=1)
        d = _minmod(qg[:, 1:-1] - qg[:, :-2], qg[:, 2:] - qg[:, 1:-1])
        qL = qg[:, 1:-2] + 0.5 * d[:, :-1]
        qR = qg[:, 2:-1] - 0.5 * d[:, 1:]
        FL, FR = flux(*qL, Brf), flux(*qR, Brf)
        UL = cons(qL[0], qL[1], qL[2], qL[3], qL[4], Brf * Brf)
        UR = cons(qR[0], qR[1], qR[2], qR[3], qR[4], Brf * Brf)
        cL, cR = _fast(qL[0], qL[3], Brf, qL[4], gam), _fast(qR[0], qR[3], Brf, qR[4], gam)
        sL = np.minimum(qL[1] - cL, qR[1] - cR)
        sR = np.maximum(qL[1] + cL, qR[1] + cR)
        Fh = np.where(sL >= 0, FL, np.where(sR <= 0, FR, (sR * FL - sL * FR + sL * sR * (UR - UL)) / (sR - sL)))
        Fw = Fh * wf
        out = -(Fw[:, 1:] - Fw[:, :-1]) / vol
        if not planar:
            rho, vr, vp, p, bp = q
            src = (2.0 * p + rho * vp * vp) * 0.5 * (edges[1:] ** 2 - edges[:-1] ** 2)
            src = src + 0.5 * C * C * (edges[:-1] ** -2.0 - edges[1:] ** -2.0)
            out[1] += src / vol[1]
        return out

    t = 0.0
    while t < t_end:
        rho, vr, vp, p, bp = prim(U)
        br = Brf[:-1] if planar else C / rc ** 2
        dt = cfl * dr / np.max(np.abs(vr) + _fast(rho, p, br, bp, gam))
        dt = min(dt, t_end - t)
        U1 = U + dt * rhs(U)
        U = 0.5 * (U + U1 + dt * rhs(U1))
        t += dt
    return rc, np.array(prim(U))
