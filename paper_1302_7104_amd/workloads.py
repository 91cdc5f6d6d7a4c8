"""Seeded synthetic workloads: problem descriptions and initial macroscopic fields.

This module is the only code shared by the HIP path's tests/benchmark and the
CPU oracle's tests.  It holds no arithmetic of the lattice Boltzmann method
itself (no equilibrium, moments or convection): it produces plain numbers —
grid sizes, radii, relaxation time, time step, boundary descriptions and the
initial fields rho, u_r, u_theta, T on the nodes — and seeded random arrays.

The problems are the annulus setups of the paper's validation section (Sec. III)
rewritten as synthetic initial-value problems:

* ``rotation``: rotational flow between coaxial cylinders (Sec. III.A), rigid
  rotation u_theta = 0.5 r at rho = 1, T = 1; ``rotation_hydrostatic`` adds the
  radial pressure balance rho = exp(omega^2 (r^2 - R1^2) / 2T).
* ``shock_tube``: radial Riemann problem (as in Sec. III.B, at laboratory radii).
* ``richtmyer_meshkov``: outward shock from Rankine-Hugoniot (Eq. Hugoniot)
  meeting a perturbed material interface (Sec. III.C).
* ``kelvin_helmholtz``: tanh shear layer with a radial-velocity perturbation
  (Eqs. KH_initial, KH_perturbation).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

# Radial boundary kinds (Sec. II.C, radial boundary condition), and the flag
# that adds the wall row's non-equilibrium part f - f^eq to the ghost layers.
WALL, INFLOW, EXTRAPOLATE = 0, 1, 2
NONEQ = 16

#: Courant number of the time-step rule, per recipe (see cfl_dt).  The
#: configurations ask for 0.3 throughout.  The combined scheme (relaxation and
#: MWB convection both taken from f(t)) amplifies the odd-even mode in r and
#: theta wherever a diagonal velocity has large Courant numbers in both
#: directions, i.e. next to the inner wall; its linearization about the
#: recipe's wall state has spectral radius 1.10 (rotation), 1.25 (shock tube)
#: and 1.08 (Kelvin-Helmholtz) at 0.3, and the FP64 runs grow seeded
#: perturbations there (the shock tube blows up within 200 steps).  Those
#: three recipes run at the largest Courant number of the ladder 0.3, 0.25,
#: 0.2 whose radius is below 0.97; Richtmyer-Meshkov (radius 0.87 at 0.3, 0.97
#: on the adjoint grid) runs as stated.
CFL = {"rotation": 0.25, "shock_tube": 0.2, "richtmyer_meshkov": 0.3, "kelvin_helmholtz": 0.25}

#: largest speed of the discrete velocity set (v_4 of Sec. II.A); used only by
#: the time-step rule below.
MAX_SPEED = 4.49


@dataclass(frozen=True)
class Problem:
    name: str
    nr: int
    nth: int
    r1: float
    r2: float
    tau: float
    dt: float
    steps: int
    bc_kind: tuple = (WALL, WALL)
    bc_par: tuple = ((0.0, 0.0, 0.0, 0.0), (0.0, 0.0, 0.0, 0.0))
    params: dict = field(default_factory=dict, compare=False, hash=False)
    nf: int = 8          # theta covers 0 < theta <= 2 pi nf / ni (nf = ni: the full annulus)
    ni: int = 8          # directions per speed: 8 octagon, 16 double, 24 triple octagon (Table I)

    @property
    def dr(self) -> float:
        return (self.r2 - self.r1) / (self.nr - 1)

    @property
    def dth(self) -> float:
        return 2.0 * math.pi * self.nf / (self.ni * self.nth)

    @property
    def nodes(self) -> int:
        return self.nr * self.nth


def cfl_dt(nr: int, nth: int, r1: float, r2: float, cfl: float = 0.3, nf: int = 8,
           ni: int = 8) -> float:
    """dt = cfl * min(dr, R1 dtheta) / max|v| (the configs' time-step rule)."""
    dr = (r2 - r1) / (nr - 1)
    dth = 2.0 * math.pi * nf / (ni * nth)
    return cfl * min(dr, r1 * dth) / MAX_SPEED


def node_coords(nr: int, nth: int, r1: float, r2: float, nf: int = 8, ni: int = 8):
    """r_i = R1 + i dr, theta_j = (j+1) dtheta with dtheta = 2 pi nf / (ni nth)
    (Sec. II.C node placement, 0-based); returns 2-D arrays R[i, j], TH[i, j]."""
    dr = (r2 - r1) / (nr - 1)
    dth = 2.0 * math.pi * nf / (ni * nth)
    r = r1 + dr * np.arange(nr, dtype=np.float64)
    th = dth * (np.arange(nth, dtype=np.float64) + 1.0)
    return np.meshgrid(r, th, indexing="ij")


def hugoniot(rho0: float, u0: float, P0: float, D: float, gamma: float = 2.0):
    """Post-shock (rho_H, u_H, P_H) behind a shock of speed D moving into the
    state (rho0, u0, P0); the solution of Eq. Hugoniot for an ideal gas with
    E = P / ((gamma - 1) rho)."""
    c0 = math.sqrt(gamma * P0 / rho0)
    M = (D - u0) / c0
    ratio = (gamma + 1.0) * M * M / ((gamma - 1.0) * M * M + 2.0)
    rhoH = rho0 * ratio
    uH = D - (D - u0) * rho0 / rhoH
    PH = P0 + rho0 * (D - u0) * (uH - u0)
    return rhoH, uH, PH


# ---------------------------------------------------------------------------
# Problem definitions.  Each returns (Problem, fields) where fields is a dict of
# float64 arrays rho, ur, ut, T of shape (nr, nth).

def rotation(nr=64, nth=128, steps=200, hydrostatic=False, omega=0.5, tau=1e-4, cfl=None):
    r1, r2 = 1.0, 2.0
    dt = cfl_dt(nr, nth, r1, r2, CFL["rotation"] if cfl is None else cfl)
    P = Problem("rotation_hydrostatic" if hydrostatic else "rotation", nr, nth, r1, r2, tau, dt,
                steps, (WALL, WALL), ((omega, 0, 0, 0), (omega, 0, 0, 0)),
                {"omega": omega})
    R, TH = node_coords(nr, nth, r1, r2)
    T = np.ones_like(R)
    rho = np.exp(omega ** 2 * (R ** 2 - r1 ** 2) / 2.0) if hydrostatic else np.ones_like(R)
    return P, dict(rho=rho, ur=np.zeros_like(R), ut=omega * R, T=T)


def shock_tube(nr=512, nth=1024, steps=2000, tau=2e-5, noise=1e-6, seed=0, cfl=None):
    r1, r2 = 0.2, 1.2
    dt = cfl_dt(nr, nth, r1, r2, CFL["shock_tube"] if cfl is None else cfl)
    P = Problem("shock_tube", nr, nth, r1, r2, tau, dt, steps, (WALL, WALL),
                ((0, 0, 0, 0), (0, 0, 0, 0)), {"seed": seed, "noise": noise})
    R, TH = node_coords(nr, nth, r1, r2)
    inner = R < 0.7
    rho = np.where(inner, 1.0, 0.125)
    T = np.where(inner, 1.0, 0.8)
    rng = np.random.default_rng(seed)
    rho = rho + noise * rng.uniform(-1.0, 1.0, size=R.shape)
    return P, dict(rho=rho, ur=np.zeros_like(R), ut=np.zeros_like(R), T=T)


RM_MODES = tuple(range(4, 17))


def rm_amplitudes(seed=1) -> np.ndarray:
    """Interface amplitudes a_k ~ U(0, 5e-3) for k = 4..16 (seeded)."""
    return np.random.default_rng(seed).uniform(0.0, 5e-3, len(RM_MODES))


def richtmyer_meshkov(nr=2048, nth=4096, steps=5000, tau=2e-5, amps=None, seed=1,
                      width=0.005, pressure_balance=False, xp=np, cfl=None):
    """Shock of Mach 2 (gamma = 2) at r = 0.8 moving outward into rho = 1,
    T = 1; interface r_I = 1.2 + sum_k a_k cos(k theta) between rho = 1 and
    rho = 3, smoothed as a tanh of width ``width``.  With pressure_balance the
    outer medium has T = 1/3 (P = 1 on both sides, as in the paper's runs);
    otherwise T = 1 on both sides.  ``amps`` may be a torch tensor (then
    xp=torch) so that the fields are differentiable in a_k."""
    r1, r2 = 0.2, 2.2
    dt = cfl_dt(nr, nth, r1, r2, CFL["richtmyer_meshkov"] if cfl is None else cfl)
    c0 = math.sqrt(2.0)
    D = 2.0 * c0
    rhoH, uH, PH = hugoniot(1.0, 0.0, 1.0, D)
    TH_ = PH / rhoH
    P = Problem("richtmyer_meshkov", nr, nth, r1, r2, tau, dt, steps, (INFLOW, WALL),
                ((rhoH, uH, 0.0, TH_), (0, 0, 0, 0)),
                {"seed": seed, "width": width, "pressure_balance": pressure_balance})
    if amps is None:
        amps = rm_amplitudes(seed)
    R, TH = node_coords(nr, nth, r1, r2)
    if xp is not np:
        import torch
        R = torch.as_tensor(R, dtype=torch.float64, device=amps.device)
        TH = torch.as_tensor(TH, dtype=torch.float64, device=amps.device)
    rI = 1.2
    for a, k in zip(amps, RM_MODES):
        rI = rI + a * xp.cos(k * TH)
    s = 0.5 * (1.0 + xp.tanh((R - rI) / width))
    rho_out, T_out = 3.0, (1.0 / 3.0 if pressure_balance else 1.0)
    shocked = R < 0.8
    one = xp.ones_like(R)
    rho = xp.where(shocked, rhoH * one, 1.0 + (rho_out - 1.0) * s)
    T = xp.where(shocked, TH_ * one, 1.0 + (T_out - 1.0) * s)
    ur = xp.where(shocked, uH * one, 0.0 * one)
    return P, dict(rho=rho, ur=ur, ut=0.0 * one, T=T)


def rm_sector(light_to_heavy=True, nr=1000, nth=450, steps=20000, shock_r=1.17, A0=0.02,
              R=1.2, k=20.0, tau=1e-5, dt=1e-5):
    """The paper's own Richtmyer-Meshkov runs (Sec. III.C): one eighth of the
    annulus R1 = 1 <= r <= R2 = 2 (N_f = 1), a shock of speed 2 moving outward
    from the light medium (rho, u_r, P) = (1, 0, 1) into the interface
    r = R + A0 cos(k R theta) (R = 1.2, A0 = 0.02, k = 20: three wavelengths
    on the sector), beyond which the medium has rho = 3 (light to heavy) or
    0.5 (heavy to light) at P = 1.  Behind the shock, inside r = shock_r (a
    reading: the paper does not place it), the Hugoniot state (1.5, 0.666667,
    0, P = 2.33333), which the inner boundary keeps supplying; the outer
    boundary extrapolates (a reading: the paper does not state it; a wall
    there reflects the transmitted shock back onto the interface, and in the
    heavy-to-light case the reflection breaks the run down before the
    amplitude recovers).  tau = dt = 1e-5 on 1000 x 450 nodes.  P = rho T
    (gamma = 2)."""
    r1, r2 = 1.0, 2.0
    rho_out = 3.0 if light_to_heavy else 0.5
    rhoH, uH, PH = hugoniot(1.0, 0.0, 1.0, 2.0)
    P = Problem("rm_sector", nr, nth, r1, r2, tau, dt, steps, (INFLOW, EXTRAPOLATE),
                ((rhoH, uH, 0.0, PH / rhoH), (0, 0, 0, 0)),
                {"light_to_heavy": light_to_heavy, "A0": A0, "R": R, "k": k,
                 "shock_r": shock_r, "shock_speed": 2.0}, 1)
    Rr, TH = node_coords(nr, nth, r1, r2, 1)
    rI = R + A0 * np.cos(k * R * TH)
    shocked = Rr < shock_r
    outer = Rr >= rI
    rho = np.where(shocked, rhoH, np.where(outer, rho_out, 1.0))
    T = np.where(shocked, PH / rhoH, np.where(outer, 1.0 / rho_out, 1.0))
    ur = np.where(shocked, uH, 0.0)
    return P, dict(rho=rho, ur=ur, ut=np.zeros_like(Rr), T=T)


def kelvin_helmholtz(nr=4096, nth=8192, steps=1000, tau=1e-5, warmup=50, cfl=None,
                     tau_equals_dt=False):
    """u_theta = 0.5 tanh((r-1)/0.01), u_r = 1e-3 sin(8 theta) exp(-((r-1)/0.02)^2),
    rho = 1, T = 1 on r in [0.5, 1.5]; walls turning with the flow at r = 0.5, 1.5."""
    r1, r2 = 0.5, 1.5
    dt = cfl_dt(nr, nth, r1, r2, CFL["kelvin_helmholtz"] if cfl is None else cfl)
    if tau_equals_dt:
        tau = dt
    w_in = 0.5 * math.tanh((r1 - 1.0) / 0.01) / r1
    w_out = 0.5 * math.tanh((r2 - 1.0) / 0.01) / r2
    P = Problem("kelvin_helmholtz", nr, nth, r1, r2, tau, dt, steps, (WALL, WALL),
                ((w_in, 0, 0, 0), (w_out, 0, 0, 0)), {"warmup": warmup})
    R, TH = node_coords(nr, nth, r1, r2)
    ut = 0.5 * np.tanh((R - 1.0) / 0.01)
    ur = 1e-3 * np.sin(8.0 * TH) * np.exp(-((R - 1.0) / 0.02) ** 2)
    return P, dict(rho=np.ones_like(R), ur=ur, ut=ut, T=np.ones_like(R))


def couette(nr=100, nth=20, steps=4000, tau=0.2, omega=(-0.1, 0.1), nf=1, dt=1e-3):
    """Flow between coaxial cylinders R1 = 1 and R2 = 2 turning at omega[0]
    and omega[1], started at rest with rho = T = 1, on the sector
    0 < theta <= 2 pi nf / 8 (Sec. III.A: 100 x 20 nodes, one eighth of the
    annulus, dt = 1e-3, tau from 0.2 down to 0.01).  The steady state tends to
    u_theta = A r + B / r (Eq. RSF)."""
    r1, r2 = 1.0, 2.0
    P = Problem("couette", nr, nth, r1, r2, tau, dt, steps, (WALL, WALL),
                ((omega[0], 0, 0, 0), (omega[1], 0, 0, 0)), {"omega": tuple(omega)}, nf)
    R, _ = node_coords(nr, nth, r1, r2, nf)
    z = np.zeros_like(R)
    return P, dict(rho=np.ones_like(R), ur=z, ut=z.copy(), T=np.ones_like(R))


def couette_profile(r, r1=1.0, r2=2.0, omega=(-0.1, 0.1)):
    """Eq. RSF: u_theta = A r + B / r with A, B from u = R omega at both walls."""
    w1, w2 = omega
    A = (w2 * r2 ** 2 - w1 * r1 ** 2) / (r2 ** 2 - r1 ** 2)
    B = r1 ** 2 * r2 ** 2 * (w1 - w2) / (r2 ** 2 - r1 ** 2)
    return A * np.asarray(r) + B / np.asarray(r)


def uniform(nr, nth, r1=1.0, r2=2.0, rho=1.0, ux=0.0, uy=0.0, T=1.0, tau=1e-3,
            bc=(WALL, WALL), bc_par=((0, 0, 0, 0), (0, 0, 0, 0)), cfl=0.3):
    """A uniform state with Cartesian velocity (ux, uy), given in polar
    components at each node."""
    dt = cfl_dt(nr, nth, r1, r2, cfl)
    P = Problem("uniform", nr, nth, r1, r2, tau, dt, 0, bc, bc_par)
    R, TH = node_coords(nr, nth, r1, r2)
    ur = ux * np.cos(TH) + uy * np.sin(TH)
    ut = -ux * np.sin(TH) + uy * np.cos(TH)
    return P, dict(rho=rho * np.ones_like(R), ur=ur, ut=ut, T=T * np.ones_like(R))


def smooth_random(nr, nth, r1=1.0, r2=2.0, tau=2e-3, seed=0, amp=0.05, cfl=0.3,
                  bc=(WALL, WALL), bc_par=((0.1, 0, 0, 0), (-0.05, 0, 0, 0)), nf=8, ni=8):
    """Smooth seeded fields: a few low azimuthal/radial modes around rho = 1,
    T = 1, u = 0, with relative amplitude ``amp``; on a sector (nf < ni) the
    azimuthal modes are periodic over the sector.  ni picks the velocity model
    (8, 16 or 24 directions per speed)."""
    rng = np.random.default_rng(seed)
    dt = cfl_dt(nr, nth, r1, r2, cfl, nf, ni)
    P = Problem("smooth_random", nr, nth, r1, r2, tau, dt, 0, bc, bc_par, {"seed": seed}, nf, ni)
    R, TH = node_coords(nr, nth, r1, r2, nf, ni)
    x = (R - r1) / (r2 - r1)
    period = float(ni) / nf

    def modes(scale):
        out = np.zeros_like(R)
        for m in range(1, 4):
            for n in range(1, 3):
                a, b, ph = rng.uniform(-1, 1, 3)
                out += scale * a * np.cos(m * period * TH + math.pi * ph) * np.sin(math.pi * n * x + b)
        return out

    rho = 1.0 + modes(amp)
    T = 1.0 + modes(amp)
    ur = modes(amp)
    ut = modes(amp)
    return P, dict(rho=rho, ur=ur, ut=ut, T=T)


def noise(shape, scale, seed) -> np.ndarray:
    """Seeded uniform noise in [-scale, scale]."""
    return scale * np.random.default_rng(seed).uniform(-1.0, 1.0, size=shape)


#: The five measured configurations, by name.
CONFIGS = {
    "rotation_64x128": lambda: rotation(64, 128, 200),
    "shock_tube_512x1024": lambda: shock_tube(512, 1024, 2000),
    "richtmyer_meshkov_2048x4096": lambda: richtmyer_meshkov(2048, 4096, 5000),
    "kelvin_helmholtz_4096x8192": lambda: kelvin_helmholtz(4096, 8192, 1000),
    "adjoint_rm_1024x2048": lambda: richtmyer_meshkov(1024, 2048, 200),
}


def reduced(make, nr, nth, steps, full=(None, None), **kw):
    """The recipe ``make`` on a smaller nr x nth grid with tau rescaled so that
    dt/tau (and the Courant numbers, which the time-step rule fixes) equal
    those of the recipe at the full size ``full`` = (nr, nth)."""
    P_full, _ = make(nr=full[0], nth=full[1], steps=1, **kw)
    P, F = make(nr=nr, nth=nth, steps=steps, **kw)
    tau = P.dt / (P_full.dt / P_full.tau)
    return replace(P, tau=tau), F
