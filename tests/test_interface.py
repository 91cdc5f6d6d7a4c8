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
    c = I.compression(t, amp, 0.02, 1.2, 1.17, 2.0)
    assert abs(c["t_meet"] - t0) < 1e-15
    assert abs(c["ratio"] - 0.7) < 1e-3
    assert abs(c["t_min"] - 0.03) < 2e-3
    assert abs(c["t_reco"] - 0.13) < 2e-3


def test_rm_sector_initial_state():
    for lth, rho_out in ((True, 3.0), (False, 0.5)):
        P, F = W.rm_sector(light_to_heavy=lth, nr=200, nth=90)
        assert P.nf == 1 and P.bc_kind == (W.INFLOW, W.WALL)
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
