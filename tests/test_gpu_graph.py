"""pclb_step_graph: n steps replayed as one captured HIP graph give the same
state as pclb_step, bit for bit, over repeated replays with eager work and
synchronisation between them, after a boundary change (which captures
again) and for odd step counts (which alternate the starting buffer)."""
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


def pair(P, F, prec):
    from paper_1302_7104_amd.sim import Sim
    sims = [Sim(P, precision=prec), Sim(P, precision=prec)]
    for s in sims:
        s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    return sims


@pytest.mark.parametrize("prec", [32, 64])
def test_graph_replays_equal_eager_steps(prec):
    P, F = W.rotation(64, 128, 200)
    eager, graph = pair(P, F, prec)
    for rep in range(4):
        eager.step(20)
        graph.step_graph(20)
        # eager work and a synchronisation between the replays
        d = graph.diagnostics_host()
        assert d[6] == 0
        assert torch.equal(eager.state, graph.state), (prec, rep)
        assert eager.steps == graph.steps == 20 * (rep + 1)
    # a boundary change takes effect in the next replay (captured again)
    for s in (eager, graph):
        s.set_bc(1, W.WALL, (0.3, 0, 0, 0))
    eager.step(20)
    graph.step_graph(20)
    assert torch.equal(eager.state, graph.state)
    # odd counts alternate the starting buffer
    for _ in range(3):
        eager.step(7)
        graph.step_graph(7)
        assert eager.current == graph.current
        assert torch.equal(eager.state, graph.state)
    graph.step_graph(0)
    assert torch.equal(eager.state, graph.state)


@pytest.mark.parametrize("prec", [32, 64])
def test_graph_replays_for_the_double_octagon_and_a_sector(prec):
    P, F = W.smooth_random(20, 128, seed=3, nf=16, ni=16)
    eager, graph = pair(P, F, prec)
    for _ in range(3):
        eager.step(5)
        graph.step_graph(5)
        torch.cuda.synchronize()
        assert torch.equal(eager.state, graph.state)
    P, F = W.smooth_random(16, 40, seed=4, nf=3)
    eager, graph = pair(P, F, prec)
    for _ in range(3):
        eager.step(4)
        graph.step_graph(4)
        assert torch.equal(eager.state, graph.state)


def test_graph_rejects_bad_counts():
    from paper_1302_7104_amd._native import PclbError
    P, F = W.rotation(16, 32, 10)
    s, _ = pair(P, F, 32)
    with pytest.raises(PclbError, match="EINVAL"):
        s.step_graph(-1)
