"""The paper's own Richtmyer-Meshkov runs (Sec. III.C, Figs. 8 and 10) on the
GPU: one eighth of the annulus, 1000 x 450 nodes, tau = dt = 1e-5, FP64, the
interface followed by markers carried with the flow.  The paper prints
A_comp / A0 = 0.715 (light to heavy; theory 0.758) and 0.65 (heavy to light;
theory 0.61), the recovery of the light-to-heavy amplitude at t = 0.13 and
the inversion of the heavy-to-light interface at t = 0.27.  These are
physics checks against printed figures (the paper's shock position and
amplitude read-out are not fully specified), held to the bounds below."""
import numpy as np
import pytest

from paper_1302_7104_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1302_7104_amd import _native
    _native.lib()          # raises if the library is missing: no fallback


def run(light_to_heavy, t_end):
    from paper_1302_7104_amd import interface as I
    from paper_1302_7104_amd.sim import Sim
    P, F = W.rm_sector(light_to_heavy=light_to_heavy)
    s = Sim(P, precision=64)
    s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    t, amp, sgn, _ = I.track_amplitude(s, P, every=20, t_end=t_end)
    d = s.diagnostics_host()
    s.close()
    assert d[6] == 0
    p = P.params
    return I.compression(t, amp, sgn, p["A0"], p["R"], p["shock_r"], p["shock_speed"])


def test_light_to_heavy():
    c = run(True, 0.17)
    print("RM light to heavy:", c)
    assert 0.70 <= c["ratio"] <= 0.85, c          # paper 0.715, theory 0.758
    assert c["t_zero"] is None
    assert c["t_reco"] is not None and 0.11 <= c["t_reco"] <= 0.15, c   # paper 0.13


def test_heavy_to_light():
    c = run(False, 0.32)
    print("RM heavy to light:", c)
    assert 0.58 <= c["ratio"] <= 0.70, c          # paper 0.65, theory 0.61
    assert c["t_zero"] is not None and 0.20 <= c["t_zero"] <= 0.30, c   # paper 0.27
