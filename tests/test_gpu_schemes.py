"""The comparison schemes (Warming-Beam, Lax-Wendroff, second-order upwind)
and the forward-Euler relaxation on the GPU, through the C ABI, against the
FP64 oracle (Sec. II.B; Sec. III.A, Figs. 5-6); the two upwind schemes on the
strip kernels against the node kernel."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1302_7104_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1302_7104_amd import _native
    _native.lib()          # raises if the library is missing: no fallback


def sim_of(P, precision, **kw):
    from paper_1302_7104_amd.sim import Sim
    return Sim(P, precision=precision, **kw)


def grid_of(P, scheme=0, relax=0):
    return O.Grid(P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, P.bc_kind, P.bc_par, nf=P.nf,
                  scheme=scheme, relax=relax)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def node_err(a, b):
    """Largest error of one node's values relative to the size of that node's
    distribution (sum over q of |f_q|): an error confined to a few nodes,
    which a norm over the whole grid can hide, shows here."""
    return float((np.abs(a - b).max(0) / np.abs(b).sum(0)).max())


NODE_TOL = {64: 1e-13, 32: 1e-6}


@pytest.mark.parametrize("relax", [0, 1])
@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_scheme_step_parity(scheme, relax):
    """Five steps of a noisy smooth state (dt/tau = 0.84, inside the stable
    range of the Euler relaxation): FP64 within 1e-12, FP32 within 2e-7."""
    P, F = W.smooth_random(33, 250, seed=21, amp=0.05, bc=(W.WALL, W.INFLOW),
                           bc_par=((0.1, 0, 0, 0), (1.05, 0.02, 0.01, 1.02)))
    g = grid_of(P, scheme, relax)
    f0 = O.init_feq(g, **F) * (1.0 + W.noise((33, P.nr, P.nth), 1e-3, 22))
    want, bad = O.step(g, f0, 5)
    assert bad == 0
    for prec, tol in ((64, 1e-12), (32, 2e-7)):
        s = sim_of(P, prec, scheme=scheme, relaxation=relax)
        s.load_state(torch.as_tensor(f0, dtype=s.dtype, device=s.device))
        s.step(5)
        got = s.state.double().cpu().numpy()
        s.close()
        assert rel(got, want) <= tol, (prec, rel(got, want))
        assert node_err(got, want) <= NODE_TOL[prec], node_err(got, want)


@pytest.mark.parametrize("scheme", [1, 2, 3])
@pytest.mark.parametrize("shape", [(21, 256), (9, 130)])
def test_schemes_on_the_strip_kernels_equal_the_node_kernel(scheme, shape):
    """The comparison schemes on the strip kernels give the node kernel's
    result bit for bit, for chunks of 1, 5 and 64 rows and the default, with
    walls and inflow at the two sides: Warming-Beam and second-order upwind
    on the FP32 kernel and, where n_theta is a multiple of 64, all three on
    the FP64 kernel (the FP32 kernel leaves Lax-Wendroff to the node kernel)."""
    from paper_1302_7104_amd import _native as N
    nr, nth = shape
    P, F = W.smooth_random(nr, nth, seed=23, amp=0.05, bc=(W.WALL, W.INFLOW),
                           bc_par=((0.1, 0, 0, 0), (1.05, 0.02, 0.01, 1.02)))
    for prec in (32, 64):
        ref = sim_of(P, prec, kernel=N.KERNEL_NODE, scheme=scheme)
        ref.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        ref.step(4)
        want = ref.state.clone()
        ref.close()
        for chunk in (0, 1, 5, 64):
            s = sim_of(P, prec, kernel=N.KERNEL_STRIP, scheme=scheme, strip_chunk=chunk)
            s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
            s.step(4)
            assert torch.equal(s.state, want), (scheme, shape, prec, chunk)
            s.close()


def test_lax_wendroff_keeps_the_node_kernel_in_fp32():
    """Lax-Wendroff's stencil reaches downwind, which the FP32 strip kernel's
    ring does not hold: asked for the strip kernel it runs on the node
    kernel."""
    from paper_1302_7104_amd import _native as N
    P, F = W.kelvin_helmholtz(16, 512, 3)
    outs = []
    for kernel in (N.KERNEL_STRIP, N.KERNEL_NODE):
        s = sim_of(P, 32, kernel=kernel, scheme=N.SCHEME_LW)
        s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        s.step(3)
        outs.append(s.state.clone())
        s.close()
    assert torch.equal(outs[0], outs[1])


def test_adjoint_refuses_comparison_schemes():
    from paper_1302_7104_amd import _native as N
    P, F = W.smooth_random(9, 64, seed=1)
    s = sim_of(P, 64, scheme=N.SCHEME_LW)
    s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    lam = torch.ones_like(s.state)
    with pytest.raises(RuntimeError):
        s.adjoint_step(s.state, lam, torch.empty_like(lam))


def test_shock_tube_schemes_on_the_gpu():
    """The shock tube at 256 x 64 for 400 steps in FP64 with each scheme: the
    density range matches the oracle's run, the MWB scheme stays inside the
    initial extremes, Warming-Beam and second-order upwind overshoot, and
    Lax-Wendroff breaks down (Fig. 6 of the paper shows its oscillations)."""
    P, F = W.shock_tube(256, 64, 400, noise=0.0)
    ranges = {}
    for scheme in range(4):
        s = sim_of(P, 64, scheme=scheme)
        s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        s.step(P.steps)
        rho = s.fields()["rho"].cpu().numpy()
        got = s.state.cpu().numpy()
        s.close()
        if scheme != 2:
            g = grid_of(P, scheme)
            want, _ = O.step(g, O.init_feq(g, **F), P.steps)
            assert rel(got, want) <= 1e-10, (scheme, rel(got, want))
        ranges[scheme] = (float(np.min(rho)), float(np.max(rho))) if np.isfinite(rho).all() else None
    print("shock tube 256x64, 400 steps, density range per scheme (MWB, WB, LW, upwind2):", ranges)
    lo, hi = ranges[0]
    assert lo >= 0.125 - 1e-6 and hi <= 1.0 + 1e-6
    for sch in (1, 3):
        assert ranges[sch][0] < 0.115 and ranges[sch][1] > 1.01
    assert ranges[2] is None or ranges[2][0] < 0.1 or ranges[2][1] > 1.1
