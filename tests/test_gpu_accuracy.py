"""Accuracy of the HIP path over whole runs: the FP64 path against the FP64
oracle at full size and full length, the FP32 error against FP64 after the
full run of every configuration, and the stability statement behind the
recipes' Courant numbers at full size."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1302_7104_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1302_7104_amd import _native
    _native.lib()          # raises if the library is missing: no fallback


def sim_of(P, precision, **kw):
    from paper_1302_7104_amd.sim import Sim
    return Sim(P, precision=precision, **kw)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def test_shock_tube_full_length_fp64_matches_oracle():
    """The shock-tube recipe at 512 x 1024 over its full 2000 steps in FP64
    against the oracle's run (stored by tests/golden/make_shock_tube_reference.py):
    all 33 distributions at 400 sample nodes, and the radial profiles of rho,
    u_r, u_theta and T (mean, min and max over theta).  Bound: 1e-12, or ten
    times the drift of the oracle against its own run perturbed by 32 ulps
    per step where the flow amplifies rounding differences more."""
    ref = np.load(os.path.join(HERE, "golden", "shock_tube_512x1024_oracle.npz"))
    P, F = W.shock_tube(512, 1024, int(ref["steps"]))
    assert P.dt == float(ref["dt"]) and P.tau == float(ref["tau"])
    s = sim_of(P, 64)
    s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    s.step(P.steps)
    nodes = ref["nodes"]
    got = s.state[:, torch.as_tensor(nodes[:, 0]), torch.as_tensor(nodes[:, 1])].cpu().numpy().T
    want = ref["f_nodes"]
    floor = rel(ref["f_nodes_noisy"], want)
    err = rel(got, want)
    fl = s.fields()
    prof = np.stack([torch.stack([x.mean(1), x.min(1).values, x.max(1).values]).cpu().numpy()
                     for x in (fl["rho"], fl["ur"], fl["ut"], fl["T"])])
    perr = np.abs(prof - ref["profiles"]).max() / np.abs(ref["profiles"]).max()
    print(f"shock tube 512x1024, 2000 steps, FP64: sampled nodes {err:.3e}, profiles {perr:.3e}, "
          f"oracle rounding-noise drift {floor:.3e}")
    bound = max(1e-12, 10 * floor)
    assert err <= bound and perr <= bound, (err, perr, floor)
    # totals (mass, two momentum components, energy), the momentum being a
    # near-cancelling sum: bounded relative to the mass
    d = s.diagnostics_host()
    dref = ref["diagnostics"][:4]
    assert np.abs(d[:4] - dref).max() <= bound * np.abs(dref).max(), (d[:4], dref)


def checkerboard_growth(cfl, steps):
    """Growth per step of a seeded odd-even perturbation (1e-9 relative) of
    the full-size Kelvin-Helmholtz recipe in FP64, and the row where it is
    largest at the end."""
    P, F = W.kelvin_helmholtz(4096, 8192, steps, cfl=cfl)
    a = sim_of(P, 64)
    a.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    b = sim_of(P, 64)
    b.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    ii = torch.arange(P.nr, device=b.device)[:, None]
    jj = torch.arange(P.nth, device=b.device)[None, :]
    b.state.mul_(1.0 + 1e-9 * (1 - 2 * ((ii + jj) % 2)).to(b.dtype))
    d0 = (b.state - a.state).abs().max().item()
    a.step(steps)
    b.step(steps)
    d = (b.state - a.state).abs()
    d1 = d.max().item()
    row = int(np.unravel_index(int(d.argmax().item()), d.shape)[1])
    del d
    a.close()
    b.close()
    torch.cuda.empty_cache()
    return (d1 / d0) ** (1.0 / steps), row


def test_kelvin_helmholtz_full_size_courant_number():
    """At 4096 x 8192 the odd-even perturbation grows at CFL 0.3 (by about 4%
    per step, in the rows next to the inner wall) and decays at the recipe's
    Courant number, as the linear analysis of the combined scheme predicts."""
    g03, row03 = checkerboard_growth(0.3, 300)
    g_cfg, _ = checkerboard_growth(None, 300)
    print(f"odd-even growth per step: CFL 0.3 {g03:.4f} (largest at row {row03}), "
          f"CFL {W.CFL['kelvin_helmholtz']} {g_cfg:.4f}")
    assert g03 > 1.02 and row03 < 16
    assert g_cfg < 1.0
