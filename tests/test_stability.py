"""The Courant number of the recipes, pinned to the stability of the combined
scheme.

The configurations ask for CFL 0.3.  The combined scheme takes the analytic
relaxation and both MWB convection terms from f(t) and adds them (Eq.
combined_scheme).  For the odd-even mode in r and theta the switch S(eta) is 0
(eta = -1), so there the convection is plain Warming-Beam (Eq. WB_Scheme_1),
whose symbol for Courant number C and wavenumber k is
    a(C, k) = |C|(1 - z) + (1/2)|C|(1 - |C|)(1 - z)^2,   z = exp(-i k sgn C).
Linearized about a uniform equilibrium, one step multiplies a Fourier mode
(k_r, k_theta) of the 33 distributions by
    G = e I + (1 - e) J - diag_q[a(C_r,q, k_r) + a(C_theta,q, k_theta)],
e = exp(-dt/tau), J the Jacobian of f -> f^eq(moments(f)) (taken here from the
oracle by central differences).  Where a diagonal velocity has large Courant
numbers in both directions (next to the inner wall, since C_theta grows as
1/r) the spectral radius of G exceeds 1: the recipes whose radius exceeds 1 at
0.3 run at a smaller Courant number.  The oracle's own runs confirm the
prediction on the shock tube.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1302_7104_amd import workloads as W

VX, VY, _ = O.velocities()


def feq_jacobian(rho, ux, uy, E, h=1e-6):
    f0 = O.feq(rho, ux, uy, E)
    J = np.zeros((33, 33))
    for q in range(33):
        e = np.zeros(33)
        e[q] = h
        J[:, q] = (O.feq(*O.macros(f0 + e)) - O.feq(*O.macros(f0 - e))) / (2 * h)
    return J


def wb_symbol(C, k):
    a = abs(C)
    z = np.exp(-1j * k * (1.0 if C >= 0 else -1.0))
    return a * (1 - z) + 0.5 * a * (1 - a) * (1 - z) ** 2


def spectral_radius(P, state, angles=np.linspace(0.0, math.pi / 4, 9),
                    ks=math.pi * np.array([0.7, 0.85, 1.0])):
    """Largest |eigenvalue| of G over the listed angles at r = R1 and the
    wavenumbers (k_r, k_theta) in ks x ks, about the equilibrium `state` =
    (rho, u_r, u_theta, T) given in polar components."""
    e = math.exp(-P.dt / P.tau)
    worst = 0.0
    for th in angles:
        ct, st = math.cos(th), math.sin(th)
        Cr = (VX * ct + VY * st) * P.dt / P.dr
        Ct = (-VX * st + VY * ct) * P.dt / (P.r1 * P.dth)
        rho, ur, ut, T = state
        J = feq_jacobian(rho, ur * ct - ut * st, ur * st + ut * ct, T)
        for kr in ks:
            for kt in ks:
                A = np.diag([wb_symbol(Cr[q], kr) + wb_symbol(Ct[q], kt) for q in range(33)])
                G = e * np.eye(33) + (1 - e) * J - A
                worst = max(worst, float(np.abs(np.linalg.eigvals(G)).max()))
    return worst


# (recipe, full size, state next to the inner wall)
CASES = {
    "rotation": (W.rotation, (64, 128), (1.0, 0.0, 0.5, 1.0)),
    "shock_tube": (W.shock_tube, (512, 1024), (1.0, 0.0, 0.0, 1.0)),
    "richtmyer_meshkov": (W.richtmyer_meshkov, (2048, 4096), (2.0, math.sqrt(2.0), 0.0, 2.5)),
    "kelvin_helmholtz": (W.kelvin_helmholtz, (4096, 8192), (1.0, 0.0, -0.5, 1.0)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_recipe_courant_number_is_linearly_stable(name):
    make, (nr, nth), state = CASES[name]
    P, _ = make(nr=nr, nth=nth, steps=1)
    P03, _ = make(nr=nr, nth=nth, steps=1, cfl=0.3)
    rho_cfg = spectral_radius(P, state)
    rho_03 = spectral_radius(P03, state)
    assert rho_cfg < 0.97, (name, rho_cfg)
    if W.CFL[name] < 0.3:
        # the recipe leaves 0.3 only where the scheme is unstable there
        assert rho_03 > 1.02, (name, rho_03)
    else:
        assert rho_03 == rho_cfg


def test_symbol_is_warming_beam_on_the_odd_even_mode():
    # the MWB term of the oracle on psi_j = (-1)^j equals a(C, pi) psi_j:
    # eta = -1 there, so S(eta) = 0 and the scheme is Warming-Beam
    for C in (0.13, 0.3, -0.27, -0.8):
        psi = np.array([1.0, -1.0, 1.0, -1.0, 1.0])
        assert abs(O.mwb_term(C, psi) - wb_symbol(C, math.pi).real) < 1e-15
        assert abs(wb_symbol(C, math.pi).imag) < 1e-15


def test_shock_tube_blows_up_at_cfl_03_and_not_at_recipe():
    """The oracle itself on the shock tube at 128 x 256 (dt/tau and Courant
    numbers of 512 x 1024): at CFL 0.3 the inner-wall region goes unstable
    (non-positive extrapolated ghost states, then non-finite values) within
    400 steps; at the recipe's Courant number it stays finite."""
    for cfl, unstable in ((0.3, True), (None, False)):
        P, F = W.reduced(lambda **k: W.shock_tube(cfl=cfl, **k), 128, 256, 400, (512, 1024))
        g = O.Grid(P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, P.bc_kind, P.bc_par, nf=P.nf)
        f, bad = O.step(g, O.init_feq(g, **F), 400)
        d = O.diagnostics(g, f)
        if unstable:
            assert bad > 0 or d[6] > 0 or not d[5] > 0
        else:
            assert bad == 0 and d[6] == 0 and d[5] > 0.4
