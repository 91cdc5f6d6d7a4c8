"""CPU checks of the device arithmetic: the per-node update, ghost layers and
adjoint that the HIP kernels share (paper_1302_7104_amd/csrc/common.h,
adjoint_node.h) are compiled for the host by tests/native/emulate.cpp and
compared with the oracle."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_1302_7104_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "emulate.cpp")
LIB = os.path.join(HERE, "native", "libemulate.so")


@pytest.fixture(scope="module")
def emu():
    csrc = os.path.join(HERE, "..", "paper_1302_7104_amd", "csrc")
    headers = [os.path.join(csrc, h) for h in ("common.h", "adjoint.h", "adjoint_node.h")] + [SRC]
    if not os.path.exists(LIB) or any(os.path.getmtime(LIB) < os.path.getmtime(h) for h in headers):
        subprocess.run(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-ffp-contract=on", "-fPIC",
                        "-shared", "-x", "hip", "--cuda-host-only", "-o", LIB, SRC], check=True)
    L = ctypes.CDLL(LIB)
    L.emu_steps.argtypes = [ctypes.c_int32, ctypes.c_int32] + [ctypes.c_double] * 4 + [
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.emu_adjoint_step.argtypes = [ctypes.c_int32, ctypes.c_int32] + [ctypes.c_double] * 4 + [
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
    return L


def run_emu(L, P, f0, steps, precision, scheme=0, relax=0):
    dt = np.float64 if precision == 64 else np.float32
    fin = np.ascontiguousarray(f0, dtype=dt)
    fout = np.empty_like(fin)
    kind = (ctypes.c_int32 * 2)(*P.bc_kind)
    par = (ctypes.c_double * 8)(*[float(x) for s in P.bc_par for x in (list(s) + [0] * 4)[:4]])
    L.emu_steps(P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, kind, par, precision,
                fin.ctypes.data, fout.ctypes.data, steps, P.nf, scheme, relax)
    return fout.astype(np.float64)


BCS = [((W.WALL, (0.2, 0, 0, 0)), (W.WALL, (-0.1, 0, 0, 0))),
       ((W.INFLOW, (1.1, 0.05, 0.02, 1.05)), (W.EXTRAPOLATE, (0, 0, 0, 0))),
       ((W.EXTRAPOLATE, (0, 0, 0, 0)), (W.INFLOW, (0.9, -0.03, 0.1, 0.95)))]


# the non-equilibrium radial boundary on both sides
BCS_NEQ = [((W.WALL | W.NONEQ, (0.2, 0, 0, 0)), (W.INFLOW | W.NONEQ, (0.9, -0.03, 0.1, 0.95))),
           ((W.EXTRAPOLATE | W.NONEQ, (0, 0, 0, 0)), (W.WALL | W.NONEQ, (-0.1, 0, 0, 0)))]


@pytest.mark.parametrize("nf", [8, 1, 3])
@pytest.mark.parametrize("bc", BCS + BCS_NEQ)
def test_emulated_device_step_matches_oracle(emu, bc, nf):
    """nf = 8 is the full annulus; 1 and 3 are sectors whose azimuthal ghosts
    rotate the direction index (Sec. II.C)."""
    P, F = W.smooth_random(9, 24, seed=3, amp=0.05, bc=(bc[0][0], bc[1][0]), bc_par=(bc[0][1], bc[1][1]),
                           nf=nf)
    g = O.Grid(P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, P.bc_kind, P.bc_par, nf=P.nf)
    f0 = O.init_feq(g, **F) * (1 + W.noise((33, P.nr, P.nth), 1e-3, 4))
    want, _ = O.step(g, f0, 4)
    got64 = run_emu(emu, P, f0, 4, 64)
    assert np.isfinite(got64).all()
    assert np.linalg.norm(got64 - want) / np.linalg.norm(want) <= 1e-13
    got32 = run_emu(emu, P, f0, 4, 32)
    assert np.isfinite(got32).all()
    assert np.linalg.norm(got32 - want) / np.linalg.norm(want) <= 1e-6


def test_emulated_recipes_finite(emu):
    for make in (W.kelvin_helmholtz, W.richtmyer_meshkov, W.shock_tube):
        P, F = make(nr=16, nth=64, steps=3)
        g = O.Grid(P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, P.bc_kind, P.bc_par, nf=P.nf)
        f0 = O.init_feq(g, **F)
        want, _ = O.step(g, f0, 3)
        got = run_emu(emu, P, f0, 3, 32)
        assert np.isfinite(got).all(), P.name
        assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-6, P.name


def run_emu_adjoint(L, P, f, lam, precision, tie):
    dt = np.float64 if precision == 64 else np.float32
    f = np.ascontiguousarray(f, dtype=dt)
    lam = np.ascontiguousarray(lam, dtype=dt)
    out = np.empty_like(f)
    kind = (ctypes.c_int32 * 2)(*P.bc_kind)
    par = (ctypes.c_double * 8)(*[float(x) for s in P.bc_par for x in (list(s) + [0] * 4)[:4]])
    L.emu_adjoint_step(P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, kind, par, precision, tie,
                       f.ctypes.data, lam.ctypes.data, out.ctypes.data, P.nf)
    return out.astype(np.float64)


@pytest.mark.parametrize("nf", [8, 1, 3])
@pytest.mark.parametrize("bc", BCS)
def test_emulated_device_adjoint_matches_oracle(emu, bc, nf):
    """The adjoint arithmetic of the kernels, run on the host, against the
    oracle's adjoint step on the same state and tie threshold, entry by entry
    relative to the entry's local scale (its size plus the largest cotangent
    around it).  At branch points of the switch (entries that move when the
    threshold moves by 1%) any of the three oracle values is accepted.  The
    rows next to each wall have a bound of their own: their stencils contain
    the ghost layers, which the device forms in its own summation order
    (FP64) or rounds to float (FP32), and a derivative of the switch near its
    tie magnifies that rounding."""
    P, F = W.smooth_random(17, 40, seed=12, amp=0.05, bc=(bc[0][0], bc[1][0]),
                           bc_par=(bc[0][1], bc[1][1]), nf=nf)
    g = O.Grid(P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, P.bc_kind, P.bc_par, nf=P.nf)
    f_or = O.init_feq(g, **F) * (1 + W.noise((33, P.nr, P.nth), 1e-2, 13))
    lam = W.noise((33, P.nr, P.nth), 1.0, 14)
    mx = np.abs(lam).max(0)
    loc = np.zeros_like(mx)
    for di in range(-2, 3):
        rows = np.clip(np.arange(P.nr) + di, 0, P.nr - 1)
        for dj in range(-2, 3):
            loc = np.maximum(loc, np.roll(mx[rows], -dj, axis=1))
    wall = np.zeros((P.nr, P.nth), bool)
    wall[:2] = wall[-2:] = True
    for prec, tie, tol, tol_wall in ((64, 1e-13, 1e-12, 1e-10), (32, 1e-6, 2e-6, 1e-3)):
        f_in = f_or.astype(np.float32).astype(np.float64) if prec == 32 else f_or
        lam_in = lam.astype(np.float32).astype(np.float64) if prec == 32 else lam
        got = run_emu_adjoint(emu, P, f_in, lam_in, prec, tie)
        w = [O.adjoint_step(g, f_in, lam_in, tie_eps=t * tie) for t in (1.0, 0.99, 1.01)]
        sc = np.abs(w[0]) + loc[None]
        branch = (np.abs(w[1] - w[0]) > 1e-9 * sc) | (np.abs(w[2] - w[0]) > 1e-9 * sc)
        err = np.where(branch, np.min([np.abs(got - x) for x in w], axis=0), np.abs(got - w[0])) / sc
        assert (err <= np.where(wall[None], tol_wall, tol)).all(), (prec, err.max())


def test_axis_columns_take_the_octant_below(emu):
    """With 8 or 16 columns every node lies on an axis theta = m pi/4, where one
    component of four directions vanishes and its computed sign is rounding
    noise.  The kernels take the upwind sides of the octant below (exact, from
    the column index); the oracle tests the sign of its rounded component.
    The term of a vanishing component carries |C| of the size of that noise,
    so the two agree to rounding."""
    for nth in (8, 16):
        P, F = W.smooth_random(9, nth, seed=5, amp=0.05, bc=(W.WALL, W.EXTRAPOLATE))
        g = O.Grid(P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, P.bc_kind, P.bc_par, nf=P.nf)
        f0 = O.init_feq(g, **F) * (1 + W.noise((33, P.nr, P.nth), 1e-3, 6))
        want, _ = O.step(g, f0, 3)
        got = run_emu(emu, P, f0, 3, 64)
        assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-14, nth


@pytest.mark.parametrize("relax", [0, 1])
@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_emulated_comparison_schemes_match_oracle(emu, scheme, relax):
    """The Warming-Beam, Lax-Wendroff and second-order upwind convection and
    the forward-Euler relaxation, as the node kernel computes them, against
    the oracle's printed forms.  tau is 2.4 dt: the forward-Euler relaxation
    amplifies by |1 - dt/tau| per step and is unstable beyond dt/tau = 2 (the
    stiffness the analytic relaxation removes)."""
    P, F = W.smooth_random(9, 24, seed=3, amp=0.05, bc=(W.WALL, W.INFLOW),
                           bc_par=((0.2, 0, 0, 0), (1.1, 0.05, 0.02, 1.05)), tau=2e-2)
    g = O.Grid(P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, P.bc_kind, P.bc_par, nf=P.nf,
               scheme=scheme, relax=relax)
    f0 = O.init_feq(g, **F) * (1 + W.noise((33, P.nr, P.nth), 1e-3, 4))
    want, _ = O.step(g, f0, 4)
    got64 = run_emu(emu, P, f0, 4, 64, scheme, relax)
    assert np.linalg.norm(got64 - want) / np.linalg.norm(want) <= 1e-13
    got32 = run_emu(emu, P, f0, 4, 32, scheme, relax)
    assert np.linalg.norm(got32 - want) / np.linalg.norm(want) <= 1e-6
    # the schemes differ from MWB (and from each other) at this size
    mwb, _ = O.step(O.Grid(P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, P.bc_kind, P.bc_par, relax=relax), f0, 4)
    assert np.linalg.norm(want - mwb) / np.linalg.norm(mwb) > 1e-6
