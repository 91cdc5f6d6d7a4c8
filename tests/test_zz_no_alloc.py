"""pclb_step_static, the entry point for callers that cannot allocate, against
pclb_step through the C ABI: bit-identical states after two calls in a row on
one GPU, the second on a smaller grid, in both precisions; and the refusal of
grids whose ghost layers exceed the static scratch array."""
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
    _native.lib()


def run(P, F, prec, n, static):
    from paper_1302_7104_amd import _native as N
    from paper_1302_7104_amd.sim import Sim
    s = Sim(P, precision=prec)
    s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    fn = s.L.pclb_step_static if static else s.L.pclb_step
    N.check(fn(s.ctx, n), s.ctx)
    torch.cuda.synchronize()
    out = s.state.cpu().numpy()
    steps = s.steps
    s.close()
    return out, steps


@pytest.mark.parametrize("prec", [32, 64])
def test_static_scratch_step_matches_step(prec):
    for nr, nth, n in ((96, 2048, 7), (40, 384, 5)):
        P, F = W.kelvin_helmholtz(nr, nth, n)
        want, _ = run(P, F, prec, n, False)
        got, steps = run(P, F, prec, n, True)
        assert steps == n
        assert np.array_equal(got, want), (prec, nr, nth)


def test_static_scratch_refuses_grids_beyond_it():
    from paper_1302_7104_amd import _native as N
    from paper_1302_7104_amd.sim import Sim
    for prec, nth in ((32, 31776), (64, 15888)):
        P, F = W.uniform(4, nth, r1=1.0, r2=2.0)
        s = Sim(P, precision=prec)
        s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        rc = s.L.pclb_step_static(s.ctx, 1)
        assert rc == -1
        assert b"static scratch" in s.L.pclb_last_error(s.ctx)
        assert s.steps == 0
        s.close()
