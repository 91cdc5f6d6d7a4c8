"""Parity of the double and triple octagon (Sec. II.A, Eq. DVM1 with N_i = 16
and 24, Table I rows 2 and 3) on the GPU with the FP64 CPU oracle, through
the C ABI: initial equilibrium, steps with every boundary kind (the
non-equilibrium one included), sectors, the comparison schemes and the
forward-Euler relaxation, fields and diagnostics.  Grids span several
256-column workgroups with a ragged last one.  Bars: FP64 normwise relative
error <= 1e-12, FP32 <= 2e-7 (the octagon's bars: the arithmetic per velocity
is the same)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1302_7104_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FP64_TOL = 1e-12
FP32_TOL = 2e-7


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1302_7104_amd import _native
    _native.lib()          # raises if the library is missing: no fallback


def grid_of(P, scheme=0, relax=0):
    return O.Grid(P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, P.bc_kind, P.bc_par, nf=P.nf, ni=P.ni,
                  scheme=scheme, relax=relax)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def node_err(a, b):
    """Largest error of one node's values relative to the size of that node's
    distribution (sum over q of |f_q|): an error confined to a few nodes,
    which a norm over the whole grid can hide, shows here."""
    return float((np.abs(a - b).max(0) / np.abs(b).sum(0)).max())


NODE_TOL = {64: 1e-13, 32: 1e-6}


def problem(ni, nf, nr, nth, bc, seed):
    return W.smooth_random(nr, nth, seed=seed, amp=0.05, bc=(bc[0][0], bc[1][0]),
                           bc_par=(bc[0][1], bc[1][1]), nf=nf, ni=ni)


def start(P, F, precision, noise_seed, scheme=0, relax=0, kernel=0):
    from paper_1302_7104_amd.sim import Sim
    s = Sim(P, precision=precision, scheme=scheme, relaxation=relax, kernel=kernel)
    s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    f = O.init_feq(grid_of(P, scheme, relax), **F)
    nz = W.noise(f.shape, 1e-3, noise_seed)
    s.state.mul_(torch.as_tensor(1.0 + nz, device=s.device, dtype=s.dtype))
    return s, f * (1.0 + nz)


BCS = [
    ((W.WALL, (0.2, 0, 0, 0)), (W.WALL, (-0.1, 0, 0, 0))),
    ((W.INFLOW, (1.1, 0.05, 0.02, 1.05)), (W.EXTRAPOLATE, (0, 0, 0, 0))),
    ((W.EXTRAPOLATE | W.NONEQ, (0, 0, 0, 0)), (W.WALL | W.NONEQ, (-0.1, 0, 0, 0))),
]


@pytest.mark.parametrize("ni", [16, 24])
def test_init_fields_and_diagnostics(ni):
    P, F = problem(ni, ni, 13, 300, BCS[0], 1)
    g = grid_of(P)
    want = O.init_feq(g, **F)
    for prec, tol in ((64, 1e-14), (32, 1e-7)):
        from paper_1302_7104_amd.sim import Sim
        s = Sim(P, precision=prec)
        s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        got = s.state.double().cpu().numpy()
        assert got.shape == (1 + 4 * ni, P.nr, P.nth)
        assert rel(got, want) <= tol, (ni, prec, rel(got, want))
        assert node_err(got, want) <= NODE_TOL[prec], node_err(got, want)
        # fields and diagnostics of the GPU's own state against the oracle's of it
        fl = s.fields()
        fw = O.fields(g, got)
        for key, w in zip(("rho", "ur", "ut", "T"), fw):
            np.testing.assert_allclose(fl[key].cpu().numpy(), w, rtol=0, atol=1e-13 * np.abs(w).max() + 1e-15)
        d = s.diagnostics_host()
        dw = O.diagnostics(g, got)
        np.testing.assert_allclose(d[:4], dw[:4], rtol=0, atol=1e-13 * abs(dw[0]))
        np.testing.assert_allclose(d[4:6], dw[4:6], rtol=1e-13)
        assert d[6] == 0
        s.close()


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("ni", [16, 24])
def test_step_parity_full_annulus(ni, bc):
    P, F = problem(ni, ni, 11, 300, bc, 2)
    want, bad = None, None
    for prec, tol in ((64, FP64_TOL), (32, FP32_TOL)):
        s, f0 = start(P, F, prec, 3)
        s.step(5)
        got = s.state.double().cpu().numpy()
        if want is None:
            want, bad = O.step(grid_of(P), f0, 5)
        assert bad == 0
        assert rel(got, want) <= tol, (ni, prec, rel(got, want))
        assert node_err(got, want) <= NODE_TOL[prec], node_err(got, want)
        s.close()


@pytest.mark.parametrize("ni,nf", [(16, 3), (24, 5), (24, 23)])
def test_step_parity_sector(ni, nf):
    """A sector 0 < theta <= 2 pi nf / ni: the azimuthal ghosts rotate the
    direction index by nf (Sec. II.C, Fig. 3)."""
    P, F = problem(ni, nf, 9, 270, BCS[1], 4)
    for prec, tol in ((64, FP64_TOL), (32, FP32_TOL)):
        s, f0 = start(P, F, prec, 5)
        s.step(6)
        got = s.state.double().cpu().numpy()
        want, bad = O.step(grid_of(P), f0, 6)
        assert bad == 0
        assert rel(got, want) <= tol, (ni, nf, prec, rel(got, want))
        assert node_err(got, want) <= NODE_TOL[prec], node_err(got, want)
        s.close()


@pytest.mark.parametrize("scheme,relax", [(1, 0), (2, 0), (3, 0), (0, 1)])
def test_step_parity_schemes_and_euler(scheme, relax):
    """The comparison schemes (Warming-Beam, Lax-Wendroff, second-order
    upwind) and the forward-Euler relaxation on the double octagon."""
    P, F = problem(16, 16, 9, 300, BCS[0], 6)
    for prec, tol in ((64, FP64_TOL), (32, FP32_TOL)):
        s, f0 = start(P, F, prec, 7, scheme, relax)
        s.step(4)
        got = s.state.double().cpu().numpy()
        want, _ = O.step(grid_of(P, scheme, relax), f0, 4)
        assert rel(got, want) <= tol, (scheme, relax, prec, rel(got, want))
        assert node_err(got, want) <= NODE_TOL[prec], node_err(got, want)
        s.close()


@pytest.mark.parametrize("ni", [16, 24])
def test_uniform_flow_stays_fixed(ni):
    """A uniform Cartesian flow with extrapolating walls is a fixed point of
    the step (its f^eq is the same at every node, so every difference and
    every relaxation term vanishes)."""
    from paper_1302_7104_amd.sim import Sim
    P, F = W.uniform(8, 300, rho=1.0, ux=0.3, uy=-0.1, T=1.0, bc=(W.EXTRAPOLATE, W.EXTRAPOLATE))
    P = W.Problem(P.name, P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, P.steps, P.bc_kind, P.bc_par,
                  P.params, ni, ni)
    s = Sim(P, precision=64)
    s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    f0 = s.state.clone()
    s.step(20)
    assert float((s.state - f0).abs().max()) <= 1e-13 * float(f0.abs().sum(0).max())


def test_allocation_free_step_matches_for_the_triple_octagon():
    from paper_1302_7104_amd.sim import Sim
    P, F = problem(24, 24, 9, 300, BCS[0], 8)
    a = Sim(P, precision=32)
    b = Sim(P, precision=32)
    for s in (a, b):
        s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    from paper_1302_7104_amd import _native as N
    a.step(3)
    N.check(b.L.pclb_step_static(b.ctx, 3), b.ctx)
    assert torch.equal(a.state, b.state)


def test_octagon_only_entry_points_refuse_larger_models():
    from paper_1302_7104_amd._native import PclbError
    from paper_1302_7104_amd.sim import Sim
    P, F = problem(16, 16, 8, 64, BCS[0], 9)
    s = Sim(P, precision=64)
    s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    with pytest.raises(PclbError, match="octagon"):
        s.noneq()
    lam = torch.zeros_like(s.state)
    out = torch.empty_like(s.state)
    with pytest.raises(PclbError, match="octagon"):
        s.adjoint_step(s.state, lam, out)


@pytest.mark.parametrize("ni", [16, 24])
@pytest.mark.parametrize("shape", [(9, 128), (21, 192), (6, 64)])
def test_strip_form_bitwise_equals_node_form(ni, shape):
    """The strip form of the double octagon (both precisions) and of the
    triple octagon (float states; its double states keep the per-node form)
    gives the per-node form's result bit for bit for chunks of 1, 5 and 64
    rows and the default: chunk tails, chunks next to both walls,
    single-strip grids and strips whose edge halo wraps around the ring."""
    from paper_1302_7104_amd import _native as N
    from paper_1302_7104_amd.sim import Sim
    nr, nth = shape
    P, F = problem(ni, ni, nr, nth, BCS[2], 10)
    for prec in ((32, 64) if ni == 16 else (32,)):
        ref = Sim(P, precision=prec, kernel=N.KERNEL_NODE)
        ref.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        ref.step(6)
        want = ref.state.cpu().numpy()
        ref.close()
        for chunk in (0, 1, 5, 64):
            s = Sim(P, precision=prec, kernel=N.KERNEL_STRIP, strip_chunk=chunk)
            s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
            s.step(6)
            got = s.state.cpu().numpy()
            s.close()
            assert np.array_equal(got, want), (ni, shape, prec, chunk)


@pytest.mark.parametrize("ni", [16, 24])
@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_strip_form_schemes_bitwise_equal_node_form(ni, scheme):
    """The comparison schemes on the strip form (Lax-Wendroff's downwind
    neighbours from the other side of the ring and the other halo) give the
    per-node form's result bit for bit; chunks of 1 and 5 rows and the
    default."""
    from paper_1302_7104_amd import _native as N
    from paper_1302_7104_amd.sim import Sim
    P, F = problem(ni, ni, 13, 192, BCS[2], 14)
    for prec in ((32, 64) if ni == 16 else (32,)):
        ref = Sim(P, precision=prec, kernel=N.KERNEL_NODE, scheme=scheme)
        ref.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        ref.step(4)
        want = ref.state.cpu().numpy()
        ref.close()
        for chunk in (0, 1, 5):
            s = Sim(P, precision=prec, kernel=N.KERNEL_STRIP, strip_chunk=chunk, scheme=scheme)
            s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
            s.step(4)
            got = s.state.cpu().numpy()
            s.close()
            assert np.array_equal(got, want), (ni, scheme, prec, chunk)


@pytest.mark.parametrize("ni", [16, 24])
def test_strip_form_parity(ni):
    """The strip kernel asked for on a grid the strip form takes (n_theta =
    256: four strips) against the oracle: the strip form for the double
    octagon and for float states of the triple, the per-node form for its
    double states."""
    from paper_1302_7104_amd import _native as N
    P, F = problem(ni, ni, 10, 256, BCS[1], 11)
    for prec, tol in ((64, FP64_TOL), (32, FP32_TOL)):
        s, f0 = start(P, F, prec, 12, kernel=N.KERNEL_STRIP)
        s.step(5)
        got = s.state.double().cpu().numpy()
        want, bad = O.step(grid_of(P), f0, 5)
        assert bad == 0
        assert rel(got, want) <= tol, (ni, prec, rel(got, want))
        assert node_err(got, want) <= NODE_TOL[prec], node_err(got, want)
        s.close()
