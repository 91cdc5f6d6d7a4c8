"""Pins of the oracle's comparison schemes and forward-Euler relaxation
(Sec. II.B; Sec. III.A, Figs. 5 and 6), each against facts that do not
restate the oracle's own formulas: exactness on polynomials, the identity
between the printed Warming-Beam form and the MWB bracket with S = 0, the
one-step return to equilibrium of the Euler relaxation at dt = tau, the
collision invariants, and the paper's shock-tube observation."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1302_7104_amd import workloads as W

SCHEMES = (O.SCHEME_MWB, O.SCHEME_WB, O.SCHEME_LW, O.SCHEME_UPWIND2)


@pytest.mark.parametrize("C", [0.9, 0.37, 0.0, -0.25, -0.8])
def test_schemes_on_polynomials(C):
    """Advection of psi(x) = x^2 by C cells: the exact new value at j = 0 is
    (0 - C)^2, so T = psi_0 - psi_0^{n+1} = -C^2 for psi_j = j^2.  Lax-Wendroff
    and Warming-Beam are exact on quadratics (second order in space and
    time); the second-order upwind scheme in forward-Euler time misses the
    C^2 term; all four are exact on linear data (T = C times the slope)."""
    j = np.arange(-2, 3, dtype=float)
    quad, lin = j ** 2, 3.0 * j + 1.0
    assert O.convection_term(O.SCHEME_LW, C, quad) == pytest.approx(-C * C, abs=1e-15)
    assert O.convection_term(O.SCHEME_WB, C, quad) == pytest.approx(-C * C, abs=1e-15)
    assert O.convection_term(O.SCHEME_UPWIND2, C, quad) == pytest.approx(0.0, abs=1e-15)
    for s in SCHEMES:
        assert O.convection_term(s, C, lin) == pytest.approx(3.0 * C, abs=1e-14), s


@pytest.mark.parametrize("C", [1.0, -1.0])
def test_unit_courant_number_is_a_shift(C):
    """At |C| = 1 the characteristic ends on a node: Lax-Wendroff,
    Warming-Beam and MWB move psi by exactly one cell."""
    psi = np.array([0.3, -1.2, 2.5, 0.7, 4.1])
    up = psi[1] if C > 0 else psi[3]
    for s in (O.SCHEME_LW, O.SCHEME_WB, O.SCHEME_MWB):
        assert psi[2] - O.convection_term(s, C, psi) == pytest.approx(up, abs=1e-15), s


def test_printed_warming_beam_is_the_bracket_with_zero_switch():
    """Eq. WB_Scheme_1 as printed equals Eq. WB_Scheme_2 with S = 0 (the
    MWB bracket without the switch), for either sign of C."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        psi = rng.normal(size=5)
        C = rng.uniform(-1, 1)
        assert O.convection_term(O.SCHEME_WB, C, psi) == pytest.approx(
            O.mwb_term(C, psi, s_mode=1), rel=1e-13, abs=1e-15)


def uniform_noisy(tau, dt, seed, nr=6, nth=16):
    P, F = W.uniform(nr, nth, rho=1.1, ux=0.2, uy=-0.1, T=0.9, tau=tau)
    g = O.Grid(P.nr, P.nth, P.r1, P.r2, tau, dt, P.bc_kind, P.bc_par, terms=1,
               relax=O.RELAX_EULER)
    f = O.init_feq(g, **F) * (1.0 + W.noise((33, nr, nth), 2e-2, seed))
    return g, f


def test_euler_relaxation_at_dt_equal_tau_reaches_equilibrium():
    """Eq. operator1_old with dt = tau is f^eq of the node's own moments in
    one step (the relaxation alone, terms = 1)."""
    g, f = uniform_noisy(1e-3, 1e-3, 5)
    out, _ = O.step(g, f, 1)
    fl = O.fields(g, f)
    want = O.init_feq(g, rho=fl[0], ur=fl[1], ut=fl[2], T=fl[3])
    np.testing.assert_allclose(out, want, rtol=1e-12, atol=1e-15)


def test_euler_relaxation_keeps_the_collision_invariants_and_is_first_order():
    """Both relaxations keep each node's mass, momentum and energy; the Euler
    form departs from the analytic one by at most (dt/tau)^2 / 2 |f - f^eq|
    (the Taylor remainder of exp(-dt/tau))."""
    tau = 1e-2
    for dt in (1e-3, 2e-3):
        g, f = uniform_noisy(tau, dt, 6)
        ga = O.Grid(g.nr, g.nth, g.r1, g.r2, tau, dt, g.bc_kind, g.bc_par, terms=1)
        eu, _ = O.step(g, f, 1)
        an, _ = O.step(ga, f, 1)
        for a, b in zip(O.fields(g, eu), O.fields(g, f)):
            np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)
        fl = O.fields(g, f)
        feq = O.init_feq(g, rho=fl[0], ur=fl[1], ut=fl[2], T=fl[3])
        bound = 0.5 * (dt / tau) ** 2 * np.abs(f - feq) + 1e-15
        assert (np.abs(eu - an) <= bound).all()
        assert (np.abs(eu - an) > 0.1 * bound).any()      # the bound is reached in order


def test_shock_tube_schemes_as_in_the_paper():
    """Sec. III.A, Fig. 6: on the shock tube the MWB scheme keeps the density
    between its initial extremes, Warming-Beam and the second-order upwind
    scheme over- and undershoot at the fronts, and Lax-Wendroff oscillates
    (here it does not survive the run).  The paper prints no numbers for
    this comparison."""
    P, F = W.shock_tube(256, 64, 400, noise=0.0)
    out = {}
    for s in SCHEMES:
        g = O.Grid(P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, P.bc_kind, P.bc_par, scheme=s)
        f, bad = O.step(g, O.init_feq(g, **F), P.steps)
        rho = O.fields(g, f)[0]
        out[s] = (bad, np.nanmin(rho) if np.isfinite(rho).all() else -np.inf,
                  np.nanmax(rho) if np.isfinite(rho).all() else np.inf)
    bad, lo, hi = out[O.SCHEME_MWB]
    assert bad == 0 and lo >= 0.125 - 1e-6 and hi <= 1.0 + 1e-6, out[O.SCHEME_MWB]
    for s in (O.SCHEME_WB, O.SCHEME_UPWIND2):
        assert out[s][1] < 0.125 - 0.01 and out[s][2] > 1.0 + 0.01, (s, out[s])
    lw = out[O.SCHEME_LW]
    assert lw[0] > 0 or lw[1] < 0.1 or lw[2] > 1.1, lw
