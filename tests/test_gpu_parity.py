"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Both sides receive the same seeded inputs from ``workloads``; the oracle
computes its own initial state.  Bars: FP64 normwise relative error
<= 1e-12; FP32 within the tolerances stated per test (FP32 storage and
convection, double collision).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1302_7104_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FP64_TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1302_7104_amd import _native
    _native.lib()          # raises if the library is missing: no fallback


def sim_of(P, precision, kernel=0, **kw):
    from paper_1302_7104_amd.sim import Sim
    return Sim(P, precision=precision, kernel=kernel, **kw)


def grid_of(P):
    return O.Grid(P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, P.bc_kind, P.bc_par, nf=P.nf)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def node_err(a, b):
    """Largest error of one node's values relative to the size of that node's
    distribution (sum over q of |f_q|): an error confined to a few nodes,
    which a norm over the whole grid can hide, shows here."""
    return float((np.abs(a - b).max(0) / np.abs(b).sum(0)).max())


NODE_TOL = {64: 1e-13, 32: 1e-6}


def start(P, F, precision, noise_seed=None, amp=1e-3, kernel=0):
    """Same initial state on both sides: f^eq(fields) times (1 + noise)."""
    s = sim_of(P, precision, kernel)
    s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    f_or = O.init_feq(grid_of(P), **F)
    if noise_seed is not None:
        nz = W.noise((33, P.nr, P.nth), amp, noise_seed)
        s.state.mul_(torch.as_tensor(1.0 + nz, device=s.device, dtype=s.dtype))
        f_or = f_or * (1.0 + nz)
    return s, f_or


def smooth_problem(nr, nth, bc, seed):
    return W.smooth_random(nr, nth, seed=seed, amp=0.05, bc=(bc[0][0], bc[1][0]),
                           bc_par=(bc[0][1], bc[1][1]))


BCS = [
    ((W.WALL, (0.2, 0, 0, 0)), (W.WALL, (-0.1, 0, 0, 0))),
    ((W.INFLOW, (1.1, 0.05, 0.02, 1.05)), (W.EXTRAPOLATE, (0, 0, 0, 0))),
    ((W.EXTRAPOLATE, (0, 0, 0, 0)), (W.INFLOW, (0.9, -0.03, 0.1, 0.95))),
]


# --------------------------------------------------------------------------
def test_init_state_matches_oracle():
    P, F = smooth_problem(37, 250, BCS[0], 1)
    for prec, tol in ((64, 1e-14), (32, 1e-7)):
        s = sim_of(P, prec)
        s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        got = s.state.double().cpu().numpy()
        want = O.init_feq(grid_of(P), **F)
        assert rel(got, want) <= tol, (prec, rel(got, want))
        assert node_err(got, want) <= NODE_TOL[prec], node_err(got, want)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("kernel", [1, 0])
def test_step_parity_fp64_small(bc, kernel):
    P, F = smooth_problem(37, 250, bc, 2)
    s, f0 = start(P, F, 64, noise_seed=3, kernel=kernel)
    s.step(5)
    got = s.state.cpu().numpy()
    want, bad = O.step(grid_of(P), f0, 5)
    assert bad == 0
    assert rel(got, want) <= FP64_TOL, rel(got, want)
    assert node_err(got, want) <= NODE_TOL[64], node_err(got, want)


BCS_NEQ = [((W.WALL | W.NONEQ, (0.2, 0, 0, 0)), (W.INFLOW | W.NONEQ, (0.9, -0.03, 0.1, 0.95))),
           ((W.EXTRAPOLATE | W.NONEQ, (0, 0, 0, 0)), (W.WALL | W.NONEQ, (-0.1, 0, 0, 0)))]


@pytest.mark.parametrize("bc", BCS_NEQ)
@pytest.mark.parametrize("kernel", [1, 0])
def test_step_parity_noneq_boundary(bc, kernel):
    """The non-equilibrium radial boundary (ghosts = f^eq of their state plus
    the wall row's f - f^eq): FP64 within 1e-12 of the oracle, FP32 within
    2e-7, on both kernels."""
    P, F = smooth_problem(37, 250, bc, 6)
    for prec, tol in ((64, FP64_TOL), (32, 2e-7)):
        s, f0 = start(P, F, prec, noise_seed=7, kernel=kernel)
        s.step(5)
        got = s.state.double().cpu().numpy()
        want, bad = O.step(grid_of(P), f0, 5)
        assert bad == 0
        assert rel(got, want) <= tol, (prec, rel(got, want))
        assert node_err(got, want) <= NODE_TOL[prec], node_err(got, want)
        s.close()


@pytest.mark.parametrize("bc", BCS)
def test_step_parity_fp32_small(bc):
    P, F = smooth_problem(37, 250, bc, 4)
    s, f0 = start(P, F, 32, noise_seed=5)
    s.step(5)
    got = s.state.double().cpu().numpy()
    want, _ = O.step(grid_of(P), f0, 5)
    assert rel(got, want) <= 2e-7, rel(got, want)
    assert node_err(got, want) <= NODE_TOL[32], node_err(got, want)


def test_rotation_config_fp64_full():
    P, F = W.rotation(64, 128, 200)
    s, f0 = start(P, F, 64)
    s.step(P.steps)
    got = s.state.cpu().numpy()
    g = grid_of(P)
    want, _ = O.step(g, f0, P.steps)
    assert rel(got, want) <= FP64_TOL, rel(got, want)
    d = s.diagnostics_host()
    dw = O.diagnostics(g, want)
    assert abs(d[0] - dw[0]) <= 1e-13 * dw[0]
    assert abs(d[3] - dw[3]) <= 1e-13 * dw[3]
    assert d[7] == P.steps


FULL = {"shock_tube": (W.shock_tube, (512, 1024)),
        "richtmyer_meshkov": (W.richtmyer_meshkov, (2048, 4096)),
        "kelvin_helmholtz": (W.kelvin_helmholtz, (4096, 8192))}


NOISE_ULPS = 32


def noise_floor(g, f0, steps, seed=0):
    """How far two FP64 oracle trajectories drift apart when one of them is
    perturbed at random by NOISE_ULPS units in the last place after every step:
    the amplification of rounding-level differences that the problem itself
    shows.  32 ulps stands for the rounding of the equilibrium, whose sums
    carry a conditioning sum|f|/rho of up to about 16 in these recipes."""
    a, _ = O.step(g, f0, steps)
    b = f0.copy()
    rng = np.random.default_rng(seed)
    for _ in range(steps):
        b, _ = O.step(g, b, 1)
        b *= 1.0 + NOISE_ULPS * 2.0 ** -52 * rng.uniform(-1.0, 1.0, b.shape)
    return a, rel(b, a)


@pytest.mark.parametrize("name", sorted(FULL))
def test_config_recipes_reduced_fp64_50_steps(name):
    """Each recipe on 128 x 256 (dt/tau and Courant numbers of its full size),
    50 steps: FP64 parity at 1e-12."""
    make, full = FULL[name]
    P, F = W.reduced(make, 128, 256, 50, full)
    s, f0 = start(P, F, 64)
    s.step(50)
    got = s.state.cpu().numpy()
    want, bad = O.step(grid_of(P), f0, 50)
    assert bad == 0
    assert rel(got, want) <= FP64_TOL, (name, rel(got, want))


@pytest.mark.parametrize("name", sorted(FULL))
def test_config_recipes_reduced_fp64_long(name):
    """300 steps of each recipe on 128 x 256.  (1) The step map on the
    recipe's own trajectory: one GPU step from each of the oracle's 300 states
    equals the oracle's next state to 1e-13 per node (scaled by the node's
    sum |f|), shocks and interfaces included.  (2) The whole run: the two
    implementations add in different orders, and a flow with shocks or shear
    layers amplifies such rounding differences over 300 steps, so the run is
    bounded by 1e-12 or by 30 times the drift between two oracle runs that
    differ by 32 ulps of random noise per step (a random walk; the ordering
    differences repeat every step and add up coherently)."""
    make, full = FULL[name]
    P, F = W.reduced(make, 128, 256, 300, full)
    g = grid_of(P)
    s, f0 = start(P, F, 64)
    s.step(300)
    got = s.state.cpu().numpy()
    want, floor = noise_floor(g, f0, 300)
    err = rel(got, want)
    # the oracle's trajectory, one step at a time on both sides
    worst = 0.0
    f = f0
    nxt = torch.empty_like(s.state)
    for _ in range(300):
        ft = torch.as_tensor(f, device=s.device)
        s.step_into(ft, nxt)
        f1, _ = O.step(g, f, 1)
        d = np.abs(nxt.cpu().numpy() - f1).max(0) / np.abs(f1).sum(0)
        worst = max(worst, float(d.max()))
        f = f1
    print(f"{name}: one step from each oracle state, max per-node error {worst:.3e}; "
          f"300-step run: GPU FP64 vs oracle {err:.3e}, oracle ulp-noise drift {floor:.3e}")
    assert np.isfinite(got).all()
    assert worst <= 1e-13, (name, worst)
    assert err <= max(FP64_TOL, 30.0 * floor), (name, err, floor)


def test_shock_tube_reduced_fp32_error():
    make, full = FULL["shock_tube"]
    P, F = W.reduced(make, 128, 256, 300, full)
    s, f0 = start(P, F, 32)
    s.step(300)
    rho = s.fields()["rho"].cpu().numpy()
    want, _ = O.step(grid_of(P), f0, 300)
    rw, _, _, Tw = O.fields(grid_of(P), want)
    err = np.abs(rho - rw) / rw
    print(f"shock tube 128x256, 300 steps: FP32 max rel density error {err.max():.3e}")
    assert err.max() <= 1e-4, err.max()


# --------------------------------------------------------------------------
# Full-size configurations, one step, in the launch configuration the
# benchmark times; the oracle evaluates sampled nodes one by one.

def sample_nodes(nr, nth, n, seed):
    rng = np.random.default_rng(seed)
    pts = [(i, j) for i in (0, 1, 2, nr - 3, nr - 2, nr - 1) for j in (0, 1, nth // 2, nth - 2, nth - 1)]
    pts += [(int(a), int(b)) for a, b in zip(rng.integers(0, nr, n), rng.integers(0, nth, n))]
    return pts


@pytest.mark.parametrize("name,prec", [
    ("kelvin_helmholtz_4096x8192", 32),
    ("richtmyer_meshkov_2048x4096", 32),
    ("shock_tube_512x1024", 64),
    ("adjoint_rm_1024x2048", 64),
])
def test_full_size_one_step_sampled(name, prec):
    P, F = W.CONFIGS[name]()
    s = sim_of(P, prec)
    s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    del F
    f0 = s.state.clone()
    s.step(1)
    nodes = sample_nodes(P.nr, P.nth, 1500, 9)
    idx_i = torch.tensor([a for a, _ in nodes], device=s.device)
    idx_j = torch.tensor([b for _, b in nodes], device=s.device)
    got = s.state[:, idx_i, idx_j].double().cpu().numpy().T
    f0h = f0.cpu().numpy()
    del f0
    s.close()
    torch.cuda.empty_cache()
    want = O.step_sample(grid_of(P), f0h, nodes)
    scale = np.abs(want).sum(1, keepdims=True)
    err = np.abs(got - want) / scale
    tol = 1e-14 if prec == 64 else 1e-6
    assert err.max() <= tol, (name, err.max())


# --------------------------------------------------------------------------
def test_bitwise_deterministic():
    P, F = W.kelvin_helmholtz(64, 384, 20)
    outs = []
    for _ in range(2):
        s = sim_of(P, 32)
        s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        s.step(20)
        outs.append(s.state.cpu().numpy().copy())
        d = s.diagnostics_host()
        outs.append(d)
    assert np.array_equal(outs[0], outs[2])
    assert np.array_equal(outs[1], outs[3])


def test_node_and_strip_kernels_bitwise_equal():
    from paper_1302_7104_amd import _native as N
    for prec in (32, 64):
        P, F = W.kelvin_helmholtz(48, 2048, 10)
        res = []
        for kernel in (N.KERNEL_NODE, N.KERNEL_STRIP):
            s = sim_of(P, prec, kernel)
            s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
            s.step(10)
            res.append(s.state.cpu().numpy())
        assert np.array_equal(res[0], res[1]), prec


@pytest.mark.parametrize("shape", [(33, 66), (12, 1024), (9, 2176), (20, 4000), (40, 250),
                                   (17, 2112), (9, 129)])
def test_strip_launch_shapes_bitwise_equal_node_kernel(shape):
    """The strip kernel in every launch shape (rows per chunk, workgroup
    order) equals the node kernel bit for bit, in both precisions: strips in
    one octant (n_theta a multiple of 1024), strips that straddle an octant
    boundary (run one thread per node), ragged last strips, a single strip,
    grids narrower than a strip and odd n_theta (node kernel), chunks of 1 to
    7 rows and of 64 (the longest), whole groups of four rows and every tail
    length."""
    from paper_1302_7104_amd import _native as N
    nr, nth = shape
    P, F = W.kelvin_helmholtz(nr, nth, 6)
    for prec in (32, 64):
        s = sim_of(P, prec, N.KERNEL_NODE)
        s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        s.step(6)
        want = s.state.cpu().numpy()
        s.close()
        for chunk, order in [(0, 1), (7, 2), (1, 1), (3, 2), (64, 1), (5, 1), (6, 2)]:
            s = sim_of(P, prec, N.KERNEL_STRIP, strip_chunk=chunk, strip_order=order)
            s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
            s.step(6)
            got = s.state.cpu().numpy()
            s.close()
            assert np.array_equal(got, want), (shape, prec, chunk, order)


@pytest.mark.parametrize("bc", BCS + BCS_NEQ)
def test_strip_kernels_bitwise_equal_node_kernel_every_boundary(bc):
    """Both strip kernels (FP32 and FP64) against the node kernel, bit for
    bit, for every radial boundary kind, the non-equilibrium ghosts included
    (the strip kernels read the ghost layers the same ghost kernel writes),
    with chunks of 3 and 64 rows and the default."""
    from paper_1302_7104_amd import _native as N
    P, F = smooth_problem(21, 192, bc, 19)
    for prec in (32, 64):
        s, _ = start(P, F, prec, noise_seed=20, kernel=N.KERNEL_NODE)
        f0 = s.state.clone()
        s.step(6)
        want = s.state.cpu().numpy()
        s.close()
        for chunk in (0, 3, 64):
            t = sim_of(P, prec, N.KERNEL_STRIP, strip_chunk=chunk)
            t.load_state(f0)
            t.step(6)
            got = t.state.cpu().numpy()
            t.close()
            assert np.array_equal(got, want), (bc, prec, chunk)


def test_init_rejects_bad_fields():
    from paper_1302_7104_amd._native import PclbError
    P, F = smooth_problem(8, 16, BCS[0], 6)
    s = sim_of(P, 64)
    rho = F["rho"].copy()
    rho[3, 4] = -1.0
    with pytest.raises(PclbError, match="EINVAL"):
        s.init_state(rho, F["ur"], F["ut"], F["T"])


def test_nonfinite_state_reported():
    from paper_1302_7104_amd._native import PclbError
    P, F = smooth_problem(8, 16, BCS[0], 7)
    s = sim_of(P, 32)
    s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    s.state[5, 2, 3] = float("nan")
    with pytest.raises(PclbError, match="ENONFINITE"):
        s.diagnostics_host()


def test_diagnostics_match_oracle():
    P, F = smooth_problem(33, 96, BCS[1], 8)
    s, f0 = start(P, F, 64, noise_seed=9)
    d = s.diagnostics_host()
    dw = O.diagnostics(grid_of(P), f0)
    np.testing.assert_allclose(d[:4], dw[:4], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(d[4:6], dw[4:6], rtol=1e-13)
    assert d[6] == 0


def test_fields_match_oracle():
    P, F = smooth_problem(33, 96, BCS[2], 10)
    s, f0 = start(P, F, 64, noise_seed=11)
    fl = s.fields()
    want = O.fields(grid_of(P), f0)
    for k, w in zip(("rho", "ur", "ut", "T"), want):
        np.testing.assert_allclose(fl[k].cpu().numpy(), w, rtol=1e-13, atol=1e-14)


# --------------------------------------------------------------------------
# Adjoint

def local_scale(w, lam):
    """Per-entry scale of an adjoint comparison: |w| plus the largest |lam|
    over all velocities in the entry's 5 x 5 neighbourhood (theta periodic),
    the size of the terms that meet in the entry."""
    m = np.abs(lam).max(0)
    out = np.zeros_like(m)
    nr = m.shape[0]
    for di in range(-2, 3):
        rows = np.clip(np.arange(nr) + di, 0, nr - 1)
        for dj in range(-2, 3):
            out = np.maximum(out, np.roll(m[rows], -dj, axis=1))
    return np.abs(w) + out[None]


@pytest.mark.parametrize("bc", BCS)
def test_adjoint_step_parity(bc):
    """One adjoint step on a noisy smooth state, both sides given the same
    state (the oracle's, rounded to the run's precision on the host) and the
    same tie threshold of the switch's derivative.

    Each entry is bounded on its own, relative to its local scale (its size
    plus the largest cotangent in its neighbourhood).  Entries whose oracle
    value moves when the tie threshold moves by 1% sit at a branch point of
    the switch: there the GPU value must equal one of the oracle values (at
    the threshold, or 1% below or above it), to the same per-entry bound.  In
    FP32 the two rows next to each wall are held to a bound of their own:
    their stencils contain the ghost layers, which the FP32 path (as its
    forward step) rounds to float and the oracle keeps in double."""
    P, F = smooth_problem(21, 70, bc, 12)
    g = grid_of(P)
    wall = np.zeros((P.nr, P.nth), bool)
    wall[:2] = wall[-2:] = True
    for prec, tie, tol, tol_wall in ((64, 1e-13, 1e-12, 1e-10), (32, 1e-6, 2e-6, 1e-3),
                                     (32, 1e-5, 2e-6, 1e-3)):
        s, f_or = start(P, F, prec, noise_seed=13, amp=1e-2)
        s.close()
        s = sim_of(P, prec, adjoint_tie=tie)
        f_in = f_or.astype(np.float32).astype(np.float64) if prec == 32 else f_or
        s.load_state(torch.as_tensor(f_in, dtype=s.dtype, device=s.device))
        lam = W.noise((33, P.nr, P.nth), 1.0, 14)
        lam_in = lam.astype(np.float32).astype(np.float64) if prec == 32 else lam
        lam_t = torch.as_tensor(lam_in, dtype=s.dtype, device=s.device).contiguous()
        out = torch.full_like(lam_t, float("nan"))    # unwritten entries stay NaN
        s.adjoint_step(s.state, lam_t, out)
        got = out.double().cpu().numpy()
        assert np.isfinite(got).all()
        w = [O.adjoint_step(g, f_in, lam_in, tie_eps=t * tie) for t in (1.0, 0.99, 1.01)]
        sc = local_scale(w[0], lam_in)
        branch = (np.abs(w[1] - w[0]) > 1e-9 * sc) | (np.abs(w[2] - w[0]) > 1e-9 * sc)
        err = np.abs(got - w[0]) / sc
        err = np.where(branch, np.min([np.abs(got - x) for x in w], axis=0) / sc, err)
        bound = np.where(wall[None], tol_wall, tol)
        print(f"precision {prec}, tie {tie:g}: branch entries {int(branch.sum())}, max error / "
              f"local scale: interior {err[:, ~wall].max():.3e}, wall rows {err[:, wall].max():.3e}")
        assert branch.sum() <= 1e-3 * branch.size, branch.sum()
        assert (err <= bound).all(), (prec, err[:, ~wall].max(), err[:, wall].max())


def test_adjoint_init_parity():
    P, F = smooth_problem(15, 40, BCS[0], 15)
    s = sim_of(P, 64)
    lam = W.noise((33, P.nr, P.nth), 1.0, 16)
    d = s.adjoint_init(torch.as_tensor(lam, device=s.device), F["rho"], F["ur"], F["ut"], F["T"])
    want = O.adjoint_init(grid_of(P), F["rho"], F["ur"], F["ut"], F["T"], lam)
    for a, b in zip(d, want):
        assert rel(a.cpu().numpy(), b) <= 1e-13


def band_weight(P):
    R, _ = W.node_coords(P.nr, P.nth, P.r1, P.r2)
    return ((R > 1.1) & (R < 1.5)) * R * P.dr * P.dth


def oracle_states(g, f0, n):
    states = [f0]
    for _ in range(n):
        states.append(O.step(g, states[-1], 1)[0])
    return states


def test_adjoint_chain_on_oracle_trajectory():
    """The GPU adjoint step applied backwards along the oracle's own FP64
    trajectory of the Richtmyer-Meshkov recipe (sharp shock, uniform regions,
    inflow and wall boundaries) reproduces the oracle's adjoint chain."""
    P, F = W.richtmyer_meshkov(24, 64, 30)
    n = 30
    g = grid_of(P)
    states = oracle_states(g, O.init_feq(g, **F), n)
    lam0 = np.broadcast_to(2.0 * states[-1].sum(0) * band_weight(P), (33, P.nr, P.nth)).copy()
    s = sim_of(P, 64)
    lam_g = torch.as_tensor(lam0, device=s.device)
    out = torch.empty_like(lam_g)
    lam_o = lam0
    for t in reversed(range(n)):
        ft = torch.as_tensor(states[t], device=s.device)
        s.adjoint_step(ft, lam_g, out)
        lam_g, out = out, lam_g
        lam_o = O.adjoint_step(g, states[t], lam_o)
    assert rel(lam_g.cpu().numpy(), lam_o) <= 1e-12, rel(lam_g.cpu().numpy(), lam_o)


def test_evolve_gradient_matches_oracle_chain():
    """Gradient of J = sum_band rho^2 r dr dtheta after n steps with respect to
    the initial density on a smooth state (no exact ties of the MWB switch):
    GPU autograd with checkpoint-recompute vs the oracle's adjoint chain."""
    from paper_1302_7104_amd.sim import Evolve, InitState
    P, F = smooth_problem(24, 64, BCS[1], 17)
    n = 30
    g = grid_of(P)
    s = sim_of(P, 64)
    rho = torch.as_tensor(F["rho"], device=s.device).requires_grad_(True)
    others = [torch.as_tensor(F[k], device=s.device) for k in ("ur", "ut", "T")]
    f0 = InitState.apply(s, rho, *others)
    fn = Evolve.apply(s, f0, n, 8)
    band = torch.as_tensor(band_weight(P), device=s.device)
    J = ((fn.sum(0) ** 2) * band).sum()
    J.backward()
    got = rho.grad.cpu().numpy()
    states = oracle_states(g, O.init_feq(g, **F), n)
    lam = np.broadcast_to(2.0 * states[-1].sum(0) * band.cpu().numpy(), (33, P.nr, P.nth)).copy()
    for t in reversed(range(n)):
        lam = O.adjoint_step(g, states[t], lam)
    want = O.adjoint_init(g, F["rho"], F["ur"], F["ut"], F["T"], lam)[0]
    assert rel(got, want) <= 1e-11, rel(got, want)


def test_evolve_checkpointing_matches_stored_trajectory():
    """Checkpoint-recompute gives bitwise the same gradient as a backward pass
    over stored states (FP32)."""
    from paper_1302_7104_amd.sim import Evolve
    P, F = W.richtmyer_meshkov(32, 96, 23)
    s = sim_of(P, 32)
    s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    f0 = s.state.clone()
    g_out = torch.as_tensor(W.noise((33, P.nr, P.nth), 1.0, 18), dtype=torch.float32, device=s.device)
    x = f0.clone().requires_grad_(True)
    Evolve.apply(s, x, 23, 5).backward(g_out)
    got = x.grad.clone()
    states = [f0.clone()]
    for _ in range(23):
        nxt = torch.empty_like(f0)
        s.step_into(states[-1], nxt)
        states.append(nxt)
    lam = g_out.clone()
    out = torch.empty_like(lam)
    for t in reversed(range(23)):
        s.adjoint_step(states[t], lam, out)
        lam, out = out, lam
    assert torch.equal(got, lam)
    # the same with every state kept by the forward (no recompute)
    x2 = f0.clone().requires_grad_(True)
    fn = Evolve.apply(s, x2, 23, 0)
    assert torch.equal(fn, states[-1])
    fn.backward(g_out)
    assert torch.equal(x2.grad, lam)


def test_evolve_keeping_every_state_checks_device_memory():
    """ckpt = 0 keeps n + 1 states: asked for more than the device holds it
    raises before allocating any of them; a negative ckpt is refused."""
    from paper_1302_7104_amd.sim import Evolve
    P, F = W.richtmyer_meshkov(32, 96, 3)
    s = sim_of(P, 64)
    s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    x = s.state.clone().requires_grad_(True)
    free, _ = torch.cuda.mem_get_info(s.device)
    n = int(2 * free // (s.state.numel() * s.state.element_size()))
    before = torch.cuda.memory_allocated(s.device)
    with pytest.raises(MemoryError, match="ckpt > 0"):
        Evolve.apply(s, x, n, 0)
    assert torch.cuda.memory_allocated(s.device) == before
    with pytest.raises(ValueError):
        Evolve.apply(s, x, 3, -1)


def test_fd_matches_fp64_adjoint_gradient():
    """dJ/da_k (J = sum_band rho^2 r dr dtheta) of the Richtmyer-Meshkov
    recipe on the 1024 x 2048 adjoint grid after 20 steps: the FP64 adjoint
    (checkpoint-recompute through the autograd function) against central
    differences of the FP64 forward with step 1e-6.  Over more steps the
    discrete map develops kinks (the MWB switch changes branch) denser than
    any practical step, and differences stop converging."""
    from paper_1302_7104_amd.sim import Evolve, InitState
    nr, nth, steps = 1024, 2048, 20
    a0 = W.rm_amplitudes(1)
    P, _ = W.richtmyer_meshkov(nr, nth, steps)
    band_np = band_weight(P)
    s = sim_of(P, 64)
    amps = torch.as_tensor(a0, device=s.device).requires_grad_(True)
    _, Ft = W.richtmyer_meshkov(nr, nth, steps, amps=amps, xp=torch)
    f0 = InitState.apply(s, Ft["rho"], Ft["ur"], Ft["ut"], Ft["T"])
    fn = Evolve.apply(s, f0, steps, 8)
    band = torch.as_tensor(band_np, device=s.device)
    J = ((fn.sum(0) ** 2) * band).sum()
    J.backward()
    g = amps.grad.detach().cpu().numpy()

    def J_of(a):
        _, F = W.richtmyer_meshkov(nr, nth, steps, amps=a)
        s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        s.step(steps)
        return float(((s.state.sum(0) ** 2) * band).sum().item())

    h = 1e-6
    fd = np.array([(J_of(a0 + h * np.eye(13)[k]) - J_of(a0 - h * np.eye(13)[k])) / (2 * h)
                   for k in range(13)])
    err = np.abs(g - fd).max() / np.abs(fd).max()
    print(f"FD (h = 1e-6) vs FP64 adjoint, 20 steps at 1024x2048: {err:.2e}")
    assert err <= 1e-4, err


@pytest.mark.xfail(strict=False, reason="over 200 steps the MWB switch changes branch at nodes whose "
                   "upwind differences cross zero for perturbations far below h = 1e-4, so central "
                   "differences do not converge to the derivative of the discrete map (measured "
                   "disagreement 1e-1 to 3e-1 at h = 1e-4, 1e-2 at h = 1e-6; 20 steps agree to 3e-5)")
def test_fd_matches_adjoint_gradient_at_the_configured_run():
    """The adjoint run as configured: Richtmyer-Meshkov on 1024 x 2048, 200
    steps, checkpoints every 20, FP64, central differences with h = 1e-4,
    target agreement 1e-4 (not reached; the measured figure is printed)."""
    from paper_1302_7104_amd.sim import Evolve, InitState
    nr, nth, steps = 1024, 2048, 200
    a0 = W.rm_amplitudes(1)
    P, _ = W.richtmyer_meshkov(nr, nth, steps)
    band_np = band_weight(P)
    s = sim_of(P, 64)
    amps = torch.as_tensor(a0, device=s.device).requires_grad_(True)
    _, Ft = W.richtmyer_meshkov(nr, nth, steps, amps=amps, xp=torch)
    f0 = InitState.apply(s, Ft["rho"], Ft["ur"], Ft["ut"], Ft["T"])
    fn = Evolve.apply(s, f0, steps, 20)
    band = torch.as_tensor(band_np, device=s.device)
    J = ((fn.sum(0) ** 2) * band).sum()
    J.backward()
    g = amps.grad.detach().cpu().numpy()

    def J_of(a):
        _, F = W.richtmyer_meshkov(nr, nth, steps, amps=a)
        s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        s.step(steps)
        return float(((s.state.sum(0) ** 2) * band).sum().item())

    h = 1e-4
    fd = np.array([(J_of(a0 + h * np.eye(13)[k]) - J_of(a0 - h * np.eye(13)[k])) / (2 * h)
                   for k in range(13)])
    err = np.abs(g - fd).max() / np.abs(fd).max()
    print(f"FD (h = 1e-4) vs FP64 adjoint, 200 steps at 1024x2048: {err:.2e}")
    assert np.isfinite(g).all() and np.abs(g).max() > 0
    assert err <= 1e-4, err


# --------------------------------------------------------------------------
# Non-equilibrium diagnostics (Sec. IV)

# order of |v| in each of the 12 components: M_2 (3), M_3 (4), M_{3,1} (2),
# M_{4,2} (3)
NONEQ_ORDER = np.array([2, 2, 2, 3, 3, 3, 3, 3, 3, 4, 4, 4])


def noneq_scale(f_nodes):
    """Size of the terms each component sums, per node: sum over q of
    |f_q| (|v_q| + |u|)^order, which bounds |f_q| |c_r|^a |c_theta|^b for the
    plain and the central velocities alike.  f_nodes: (n, 33) -> (n, 12)."""
    vx, vy, _ = O.velocities()
    f_nodes = np.asarray(f_nodes, dtype=np.float64)
    rho = f_nodes.sum(1)
    u = np.hypot(f_nodes @ vx, f_nodes @ vy) / rho
    base = np.hypot(vx, vy)[None, :] + u[:, None]                     # (n, 33)
    return np.stack([(np.abs(f_nodes) * base ** p).sum(1) for p in NONEQ_ORDER], axis=1)


@pytest.mark.parametrize("prec", [64, 32])
def test_noneq_matches_oracle(prec):
    from paper_1302_7104_amd import _native as N
    P, F = smooth_problem(33, 130, BCS[2], 12)
    s, _ = start(P, F, prec, noise_seed=13, amp=2e-2)
    f = s.state.double().cpu().numpy()
    want = O.noneq(grid_of(P), f)
    got = s.noneq().cpu().numpy()
    scale = noneq_scale(f.reshape(33, -1).T).T.reshape(1, 12, P.nr, P.nth)
    assert float(np.max(np.abs(got - want) / scale)) <= 1e-14
    # a subset of kinds keeps the order M, M*, Delta, Delta*
    sub = s.noneq(N.NONEQ_DSTAR | N.NONEQ_M).cpu().numpy()
    np.testing.assert_array_equal(sub[0], got[0])
    np.testing.assert_array_equal(sub[1], got[3])
    # an explicit state argument, not the simulation's own
    other = s.state * 1.01
    oh = other.double().cpu().numpy()
    want_o = O.noneq(grid_of(P), oh)[0]
    got_o = s.noneq(N.NONEQ_M, other).cpu().numpy()[0]
    scale_o = noneq_scale(oh.reshape(33, -1).T).T.reshape(12, P.nr, P.nth)
    assert float(np.max(np.abs(got_o - want_o) / scale_o)) <= 1e-14


def test_noneq_rejects_empty_kind_set():
    from paper_1302_7104_amd import _native as N
    P, F = smooth_problem(9, 64, BCS[0], 1)
    s, _ = start(P, F, 64)
    with pytest.raises(RuntimeError):
        s.noneq(0)
    with pytest.raises(RuntimeError):
        s.noneq(N.NONEQ_ALL + 1)


def test_noneq_full_size_sampled():
    P, F = W.CONFIGS["kelvin_helmholtz_4096x8192"]()
    s = sim_of(P, 32)
    s.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    del F
    s.step(20)
    nodes = sample_nodes(P.nr, P.nth, 1000, 14)
    got = s.noneq()
    idx_i = torch.tensor([a for a, _ in nodes], device=s.device)
    idx_j = torch.tensor([b for _, b in nodes], device=s.device)
    got = got[:, :, idx_i, idx_j].cpu().numpy().transpose(2, 0, 1)      # (node, kind, comp)
    fh = s.state.cpu().numpy()
    s.close()
    torch.cuda.empty_cache()
    want = O.noneq_sample(grid_of(P), fh, nodes)
    f_nodes = np.stack([fh[:, a, b] for a, b in nodes])
    scale = noneq_scale(f_nodes)[:, None, :]
    assert float(np.max(np.abs(got - want) / scale)) <= 1e-14
