"""Whole-grid FP64 parity at the full sizes of the two largest
configurations: the first 50 steps of the Richtmyer-Meshkov run on
2048 x 4096 and the first 5 steps of the Kelvin-Helmholtz run on 4096 x 8192,
every node of every velocity against the oracle run on the host (which takes
tens of seconds at these sizes), in the launch configuration the benchmark
times (the FP64 strip kernel)."""
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


def run_both(P, F, steps):
    from paper_1302_7104_amd.sim import Sim
    g = O.Grid(P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, P.bc_kind, P.bc_par, nf=P.nf)
    f0 = O.init_feq(g, **F)
    s = Sim(P, precision=64)
    s.load_state(torch.as_tensor(f0, device=s.device))
    del f0
    s.step(steps)
    got = s.state.cpu().numpy()
    s.close()
    torch.cuda.empty_cache()
    want, bad = O.step(g, O.init_feq(g, **F), steps)
    assert bad == 0
    return got, want


def errors(got, want):
    d = got - want
    norm = float(np.sqrt((d * d).sum() / (want * want).sum()))
    node = float((np.abs(d).max(0) / np.abs(want).sum(0)).max())
    return norm, node


def test_richtmyer_meshkov_full_size_first_50_steps():
    P, F = W.richtmyer_meshkov(2048, 4096, 50)
    got, want = run_both(P, F, 50)
    norm, node = errors(got, want)
    print(f"Richtmyer-Meshkov 2048x4096, 50 FP64 steps: norm {norm:.3e}, per node {node:.3e}")
    assert norm <= 1e-12, norm
    assert node <= 1e-12, node


def test_kelvin_helmholtz_full_size_first_5_steps():
    P, F = W.kelvin_helmholtz(4096, 8192, 5)
    got, want = run_both(P, F, 5)
    norm, node = errors(got, want)
    print(f"Kelvin-Helmholtz 4096x8192, 5 FP64 steps: norm {norm:.3e}, per node {node:.3e}")
    assert norm <= 1e-12, norm
    assert node <= 1e-13, node
