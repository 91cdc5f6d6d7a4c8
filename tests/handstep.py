"""Arbitrary-precision hand stepper for tiny grids (test infrastructure).

A third, deliberately different implementation of one combined-scheme step
(Sec. II.B of Lin et al., Eq. combined_scheme), written in pure Python with
mpmath at 50 significant digits, using the paper's 1-based indices
(i_r = 1..N_r, i_theta = 1..N_theta; ghosts i_r in {-1, 0, N_r+1, N_r+2}) and
the paper's eta-form of the MWB switch.  It is used only to pin the FP64
oracle on grids of a few nodes, where its cost (a second or so per step) is
acceptable.  It imports nothing from the oracle or from the HIP package.
"""
from __future__ import annotations

import mpmath as mp

mp.mp.dps = 50

SPEEDS = [mp.mpf(0), mp.mpf(1), mp.mpf("2.92"), mp.mpf("2.99"), mp.mpf("4.49")]
NI = 8
B0, B1, B2, B3, B4 = mp.mpf(8), mp.mpf(-1) / 4, mp.mpf(1), mp.mpf(-6), mp.mpf(48)


def velocity_list():
    """[(k, i, vx, vy)] in the order q = 0 (rest), then k = 1..4, i = 1..8."""
    out = [(0, 0, mp.mpf(0), mp.mpf(0))]
    for k in range(1, 5):
        for i in range(1, NI + 1):
            ang = 2 * mp.pi * (i - 1) / NI
            out.append((k, i, SPEEDS[k] * mp.cos(ang), SPEEDS[k] * mp.sin(ang)))
    return out


VEL = velocity_list()


def _mod(a, b):
    return a if a <= b else a - b


def weight(k, E):
    """Eqs. F_k / F_0 with the octagon row of Table I."""
    if k == 0:
        return 1 - B0 * sum(weight(kk, E) for kk in range(1, 5))
    x = [s * s for s in SPEEDS]
    o = [_mod(k + l, 4) for l in (1, 2, 3)]
    a, b, c = x[o[0]], x[o[1]], x[o[2]]
    den = x[k] * (x[k] - a) * (x[k] - b) * (x[k] - c)
    num = B4 * E ** 4 + B3 * (a + b + c) * E ** 3 + B2 * (a * b + b * c + c * a) * E ** 2 + B1 * a * b * c * E
    return num / den


def equilibrium(rho, ux, uy, E):
    """Eq. feq for all 33 velocities."""
    Fk = [weight(k, E) for k in range(5)]
    u2 = ux * ux + uy * uy
    res = []
    for (k, i, vx, vy) in VEL:
        w = vx * ux + vy * uy
        g = 1 - u2 / (2 * E)
        br = (1 - u2 / (2 * E) + u2 ** 2 / (8 * E ** 2)) + w / E * g + w ** 2 / (2 * E ** 2) * g \
            + w ** 3 / (6 * E ** 3) + w ** 4 / (24 * E ** 4)
        res.append(rho * Fk[k] * br)
    return res


def hydro(fnode):
    """Eqs. moment1-3 for one node -> (rho, ux, uy, E)."""
    rho = sum(fnode)
    ux = sum(f * v[2] for f, v in zip(fnode, VEL)) / rho
    uy = sum(f * v[3] for f, v in zip(fnode, VEL)) / rho
    E = sum(f * ((v[2] - ux) ** 2 + (v[3] - uy) ** 2) / 2 for f, v in zip(fnode, VEL)) / rho
    return rho, ux, uy, E


def mwb(C, m2, m1, c0, p1, p2):
    """[C + C(1-|C|)(1-S(eta))(1-eta)/2] delta with the upwind choice of Sec. II.B."""
    if C >= 0:
        delta, top = c0 - m1, m1 - m2
    else:
        delta, top = p1 - c0, p2 - p1
    if delta == 0:
        return mp.mpf(0)
    eta = top / delta
    S = (abs(eta) - 1) / (abs(eta) + 1)
    return (C + C * (1 - abs(C)) * (1 - S) * (1 - eta) / 2) * delta


def step(f, Nr, Nt, R1, R2, tau, dt, bc):
    """One step.  f: dict (q, ir, it) -> mpf with 1-based ir, it.
    bc: [(kind, params) inner, (kind, params) outer], kinds 'wall', 'inflow',
    'extrapolate' as in Sec. II.C (radial boundary condition)."""
    tau, dt = mp.mpf(tau), mp.mpf(dt)
    dr = (mp.mpf(R2) - mp.mpf(R1)) / (Nr - 1)
    dth = 2 * mp.pi / Nt
    rad = lambda ir: mp.mpf(R1) + (ir - 1) * dr
    ang = lambda it: it * dth
    Q = len(VEL)
    g = dict(f)
    # azimuthal ghosts (N_f = N_i: same velocity index)
    for q in range(Q):
        for ir in range(1, Nr + 1):
            for it in (-1, 0):
                g[(q, ir, it)] = f[(q, ir, Nt + it)]
            for it in (Nt + 1, Nt + 2):
                g[(q, ir, it)] = f[(q, ir, it - Nt)]
    H = {}
    for ir in range(1, Nr + 1):
        for it in range(1, Nt + 1):
            H[(ir, it)] = hydro([f[(q, ir, it)] for q in range(Q)])
    # radial ghosts
    for side, (kind, par) in enumerate(bc):
        par = [mp.mpf(p) for p in par]
        for it in range(1, Nt + 1):
            th = ang(it)
            ct, st = mp.cos(th), mp.sin(th)
            if side == 0:
                a, b, gh = H[(1, it)], H[(2, it)], (0, -1)
            else:
                a, b, gh = H[(Nr, it)], H[(Nr - 1, it)], (Nr + 1, Nr + 2)
            rho_prev, rho_pp = a[0], b[0]
            T_prev, T_pp = a[3], b[3]
            ur = lambda h: h[1] * ct + h[2] * st
            ut = lambda h: -h[1] * st + h[2] * ct
            ur_prev, ur_pp, ut_prev, ut_pp = ur(a), ur(b), ut(a), ut(b)
            for ghost in gh:
                rho_g = 2 * rho_prev - rho_pp
                T_g = 2 * T_prev - T_pp
                ur_g = 2 * ur_prev - ur_pp
                ut_g = 2 * ut_prev - ut_pp
                rho_pp, rho_prev = rho_prev, rho_g
                T_pp, T_prev = T_prev, T_g
                ur_pp, ur_prev = ur_prev, ur_g
                ut_pp, ut_prev = ut_prev, ut_g
                if kind == "wall":
                    vr, vt = mp.mpf(0), par[0] * rad(ghost)
                elif kind == "inflow":
                    rho_g, vr, vt, T_g = par
                else:
                    vr, vt = ur_g, ut_g
                ux = vr * ct - vt * st
                uy = vr * st + vt * ct
                fe = equilibrium(rho_g, ux, uy, T_g)
                for q in range(Q):
                    g[(q, ghost, it)] = fe[q]
    e = mp.exp(-dt / tau)
    out = {}
    for ir in range(1, Nr + 1):
        r = rad(ir)
        for it in range(1, Nt + 1):
            rho, ux, uy, E = H[(ir, it)]
            fe = equilibrium(rho, ux, uy, E)
            th = ang(it)
            ct, st = mp.cos(th), mp.sin(th)
            for q, (k, i, vx, vy) in enumerate(VEL):
                vr = vx * ct + vy * st
                vt = -vx * st + vy * ct
                Cr = vr * dt / dr
                Ct = vt * dt / (r * dth)
                val = fe[q] + (g[(q, ir, it)] - fe[q]) * e
                val -= mwb(Cr, *(g[(q, ir + d, it)] for d in (-2, -1, 0, 1, 2)))
                val -= mwb(Ct, *(g[(q, ir, it + d)] for d in (-2, -1, 0, 1, 2)))
                out[(q, ir, it)] = val
    return out
