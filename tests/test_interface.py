"""Host-side pieces of the Richtmyer-Meshkov analysis: the bilinear
interpolation the interface markers use, the compression read-out, and the
sector recipe's initial state (Hugoniot state behind the shock, pressure
balance across the interface, three wavelengths on the sector)."""
import numpy as np

from paper_1302_7104_amd import interface as I
from paper_1302_7104_amd import workloads as W


def test_bilinear_interpolation_is_exact_on_bilinear_fields():
    nr, nth, r1, dr, dth = 30, 40, 1.0, 0.01, 0.02
    i = np.arange(nr)[:, None]
    j = np.arange(nth)[None, :]
    field = 2.0 + 3.0 * i + 0.5 * j + 0.25 * i * j     # bilinear in (i, j)
    rng = np.random.default_rng(1)
    x = rng.uniform(0, nr - 1, 200)
    y = rng.uniform(0, nth - 1, 200)
    got = I._interp(field, r1 + x * dr, (y + 1.0) * dth, r1, dr, dth)
    np.testing.assert_allclose(got, 2.0 + 3.0 * x + 0.5 * y + 0.25 * x * y, rtol=1e-13)
    # periodic in theta: column -1 is the last column
    f2 = np.tile(np.arange(nth, dtype=float), (nr, 1))
    got = I._interp(f2, np.full(3, r1), np.array([0.5, 0.25, 0.75]) * dth, r1, dr, dth)
    np.testing.assert_allclose(got, [(nth - 1) * 0.5, (nth - 1) * 0.75, (nth - 1) * 0.25])


def test_compression_readout():
    t = np.linspace(0, 0.5, 501)
    t0 = (1.2 - 0.02 - 1.17) / 2.0
    # amplitude: 0.02 until the shock, down to 0.014 at t0 + 0.03, then up
    amp = np.where(t < t0, 0.02, np.where(t < t0 + 0.03, 0.02 - 0.2 * (t - t0),
                                          0.014 + 0.06 * (t - t0 - 0.03)))
    c = I.compression(t, amp, amp, 0.02, 1.2, 1.17, 2.0)
    assert abs(c["t_meet"] - t0) < 1e-15
    assert abs(c["ratio"] - 0.7) < 1e-3
    assert abs(c["t_min"] - 0.03) < 2e-3
    assert abs(c["t_reco"] - 0.13) < 2e-3
    assert c["t_zero"] is None
    # an inverting interface: the signed amplitude falls through zero at
    # t0 + 0.2 and grows back to -A0 by t0 + 0.4
    sg = np.where(t < t0, 0.02, 0.02 - 0.1 * (t - t0))
    c = I.compression(t, np.abs(sg), sg, 0.02, 1.2, 1.17, 2.0)
    assert abs(c["t_zero"] - 0.2) < 1e-9
    assert abs(c["t_reco"] - 0.4) < 2e-3


def test_rm_sector_initial_state():
    for lth, rho_out in ((True, 3.0), (False, 0.5)):
        P, F = W.rm_sector(light_to_heavy=lth, nr=200, nth=90)
        assert P.nf == 1 and P.bc_kind == (W.INFLOW, W.EXTRAPOLATE)
        R, TH = W.node_coords(P.nr, P.nth, P.r1, P.r2, P.nf)
        inner, outer = R < 1.17, R > 1.25
        np.testing.assert_allclose(F["rho"][inner], 1.5)
        np.testing.assert_allclose(F["ur"][inner], 2.0 / 3.0, rtol=1e-12)
        np.testing.assert_allclose((F["rho"] * F["T"])[inner], 7.0 / 3.0, rtol=1e-12)
        np.testing.assert_allclose(F["rho"][outer], rho_out)
        np.testing.assert_allclose((F["rho"] * F["T"])[R > 1.17], 1.0)     # pressure balance
        # the interface completes whole wavelengths on the sector: the
        # first and last columns see the same radius pattern shifted by one
        # column spacing
        r_i = 1.2 + 0.02 * np.cos(24.0 * TH[0])
        assert abs(np.cos(24.0 * 2 * np.pi / 8) - 1.0) < 1e-12
        assert r_i.max() <= 1.22 and r_i.min() >= 1.18


def _riemann_contact_velocity(left, right, gamma=2.0):
    """Velocity of the contact in the exact Riemann solution of an ideal gas
    between the states left and right = (rho, u, P) (pressure function of
    the two nonlinear waves, bisection)."""
    def f(p, rho, pk):
        c = np.sqrt(gamma * pk / rho)
        if p > pk:                                     # shock
            A, B = 2.0 / ((gamma + 1.0) * rho), (gamma - 1.0) / (gamma + 1.0) * pk
            return (p - pk) * np.sqrt(A / (p + B))
        return 2.0 * c / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
    (rl, ul, pl), (rr, ur, pr) = left, right
    lo, hi = 1e-9, 1e3
    for _ in range(200):
        p = 0.5 * (lo + hi)
        if f(p, rl, pl) + f(p, rr, pr) + ur - ul > 0:
            hi = p
        else:
            lo = p
    return 0.5 * (ul + ur) + 0.5 * (f(p, rr, pr) - f(p, rl, pl))


def test_theory_compression_ratios_as_printed():
    """Sec. III.C quotes the theoretical compression ratios 1 - du/D of its two
    runs as 0.758 (light to heavy) and 0.61 (heavy to light), du being the
    velocity the interface takes when the shock of speed D = 2 has crossed
    it.  From the recipe's states (the Hugoniot state behind the shock, the
    media at rest at P = 1) the exact Riemann solution gives the same."""
    for lth, printed, tol in ((True, 0.758, 3e-3), (False, 0.61, 2e-3)):
        P, F = W.rm_sector(light_to_heavy=lth, nr=200, nth=90)
        rho_h, u_h, T_h = P.bc_par[0][0], P.bc_par[0][1], P.bc_par[0][3]
        rho_out = 3.0 if lth else 0.5
        du = _riemann_contact_velocity((rho_h, u_h, rho_h * T_h), (rho_out, 0.0, 1.0))
        assert abs((1.0 - du / P.params["shock_speed"]) - printed) <= tol, (lth, 1.0 - du / 2.0)
