"""Python wrapper of the FP64 CPU oracle (``pclb_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the HIP library; the two only meet in the tests, which feed both the same
seeded inputs.

Every function here is a thin ctypes call into the plain C++ implementation of
the method of Lin et al., "Polar coordinate lattice Boltzmann modeling of
compressible flows" (Sec. II); the docstrings name the passage each follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pclb_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

NQ = 33
WALL, INFLOW, EXTRAPOLATE = 0, 1, 2
NONEQ = 16     # flag: ghost layers add the wall row's f - f^eq
# convection schemes and relaxation forms (Sec. II.B; Sec. III.A, Figs. 5-6)
SCHEME_MWB, SCHEME_WB, SCHEME_LW, SCHEME_UPWIND2 = 0, 1, 2, 3
RELAX_ANALYTIC, RELAX_EULER = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (portable flags: the library travels to
    other hosts, so no -march=native; no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC",
               "-shared", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _OrGrid(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int32), ("nth", ctypes.c_int32),
                ("r1", ctypes.c_double), ("r2", ctypes.c_double),
                ("tau", ctypes.c_double), ("dt", ctypes.c_double),
                ("bc_kind", ctypes.c_int32 * 2),
                ("bc_par", (ctypes.c_double * 4) * 2),
                ("terms", ctypes.c_int32), ("nf", ctypes.c_int32),
                ("scheme", ctypes.c_int32), ("relax", ctypes.c_int32),
                ("ni", ctypes.c_int32)]


@dataclass
class Grid:
    """Annulus R1 <= r <= R2 with nr x nth nodes, relaxation time tau, step dt
    and one radial boundary description per side (0 inner, 1 outer)."""
    nr: int
    nth: int
    r1: float
    r2: float
    tau: float
    dt: float
    bc_kind: tuple = (WALL, WALL)
    bc_par: tuple = ((0.0, 0.0, 0.0, 0.0), (0.0, 0.0, 0.0, 0.0))
    terms: int = 7
    nf: int = 8           # theta covers 2 pi nf / 8 (Sec. II.C); 8 = full annulus
    scheme: int = 0       # SCHEME_MWB, SCHEME_WB, SCHEME_LW, SCHEME_UPWIND2
    relax: int = 0        # RELAX_ANALYTIC (Eq. operator1_new), RELAX_EULER (Eq. operator1_old)
    ni: int = 8           # directions per speed: 8, 16, 24 (Table I); nf counts in units of 2 pi / ni

    @property
    def nq(self) -> int:
        return 1 + 4 * int(self.ni)

    def c(self) -> _OrGrid:
        if int(self.ni) not in (8, 16, 24):
            raise ValueError("ni must be 8, 16 or 24")
        if not 1 <= int(self.nf) <= int(self.ni):
            raise ValueError("nf must be in 1..ni")
        g = _OrGrid()
        g.nr, g.nth = self.nr, self.nth
        g.r1, g.r2, g.tau, g.dt = self.r1, self.r2, self.tau, self.dt
        for s in range(2):
            g.bc_kind[s] = int(self.bc_kind[s])
            p = list(self.bc_par[s]) + [0.0] * (4 - len(self.bc_par[s]))
            for a in range(4):
                g.bc_par[s][a] = float(p[a])
        g.terms = self.terms
        g.nf = int(self.nf)
        g.scheme = int(self.scheme)
        g.relax = int(self.relax)
        g.ni = int(self.ni)
        return g


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    if _lib is None:
        path = build(force=False)
        L = ctypes.CDLL(path)
        G = ctypes.POINTER(_OrGrid)
        L.or_velocities.argtypes = [_D, _D, _I]
        L.or_weights.argtypes = [ctypes.c_double, ctypes.c_int32, _D]
        L.or_feq.argtypes = [ctypes.c_double] * 4 + [_D]
        L.or_macros.argtypes = [_D, _D]
        L.or_relax_node.argtypes = [_D, ctypes.c_double, ctypes.c_double, _D]
        L.or_mwb_term.argtypes = [ctypes.c_double, _D, ctypes.c_int32]
        L.or_mwb_term.restype = ctypes.c_double
        L.or_mwb_term_eta.argtypes = [ctypes.c_double, _D]
        L.or_convection_term.argtypes = [ctypes.c_int32, ctypes.c_double, _D]
        L.or_convection_term.restype = ctypes.c_double
        L.or_mwb_term_eta.restype = ctypes.c_double
        L.or_mwb_grad.argtypes = [ctypes.c_double, _D, ctypes.c_double, _D]
        L.or_step.argtypes = [G, _D, _D, ctypes.c_int32]
        L.or_step.restype = ctypes.c_int
        L.or_step_sample.argtypes = [G, _D, _I, ctypes.c_int32, _D]
        L.or_init_feq.argtypes = [G, _D, _D, _D, _D, _D]
        L.or_fields.argtypes = [G, _D, _D, _D, _D, _D]
        L.or_diagnostics.argtypes = [G, _D, _D]
        L.or_adjoint_step.argtypes = [G, _D, _D, ctypes.c_double, _D]
        L.or_adjoint_step.restype = ctypes.c_int
        L.or_adjoint_init.argtypes = [G, _D, _D, _D, _D, _D, _D, _D, _D, _D]
        L.or_noneq.argtypes = [G, _D, _D]
        L.or_noneq_sample.argtypes = [G, _D, _I, ctypes.c_int32, _D]
        L.or_num_threads.restype = ctypes.c_int
        L.or_set_threads.argtypes = [ctypes.c_int32]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def velocities():
    """Eq. DVM1 with the speeds of Sec. II.A: (vx[33], vy[33], k[33])."""
    vx = np.zeros(NQ); vy = np.zeros(NQ); k = np.zeros(NQ, dtype=np.int32)
    lib().or_velocities(_p(vx), _p(vy), k.ctypes.data_as(_I))
    return vx, vy, k


def weights(E: float, row: int = 0) -> np.ndarray:
    """Eqs. F_k with Table I row ``row`` (0 octagon, 1 double, 2 triple)."""
    F = np.zeros(5)
    lib().or_weights(float(E), int(row), _p(F))
    return F


def feq(rho, ux, uy, E) -> np.ndarray:
    """Eq. feq for one state; returns the 33 equilibrium values."""
    out = np.zeros(NQ)
    lib().or_feq(float(rho), float(ux), float(uy), float(E), _p(out))
    return out


def macros(f33) -> np.ndarray:
    """Eqs. moment1-moment3 for one node: (rho, u_x, u_y, E)."""
    f33 = _f64(f33); out = np.zeros(4)
    lib().or_macros(_p(f33), _p(out))
    return out


def relax_node(f33, dt, tau) -> np.ndarray:
    """Eq. operator1_new for one node."""
    f33 = _f64(f33); out = np.zeros(NQ)
    lib().or_relax_node(_p(f33), float(dt), float(tau), _p(out))
    return out


#: tie threshold of the adjoint for states computed in double precision
TIE_FP64 = 1e-13


def convection_term(scheme: int, C, psi5) -> float:
    """psi_j^n - psi_j^{n+1} of one sweep of the given scheme (SCHEME_*) for
    psi_{j-2..j+2} at Courant number C."""
    psi5 = _f64(psi5)
    return lib().or_convection_term(int(scheme), float(C), _p(psi5))


def mwb_term(C, psi5, s_mode: int = 0) -> float:
    """Eq. MWB Scheme (division-free form of the switch): the convection term
    for psi_{j-2..j+2} at Courant number C.  s_mode=1 sets S = 0 (Warming-Beam)."""
    psi5 = _f64(psi5)
    return lib().or_mwb_term(float(C), _p(psi5), int(s_mode))


def mwb_term_eta(C, psi5) -> float:
    """The same term with eta and S(eta) as printed (0 when delta = 0)."""
    psi5 = _f64(psi5)
    return lib().or_mwb_term_eta(float(C), _p(psi5))


def mwb_grad(C, psi5, tie_eps: float = TIE_FP64) -> np.ndarray:
    """d(mwb_term)/d(psi_{j-2..j+2}) with the derivative convention at the
    kinks: differences within tie_eps x the stencil magnitude count as zero,
    sgn(0) = 0, and (1, 0) where both upwind differences vanish."""
    psi5 = _f64(psi5); g = np.zeros(5)
    lib().or_mwb_grad(float(C), _p(psi5), float(tie_eps), _p(g))
    return g


def step(grid: Grid, f: np.ndarray, nsteps: int) -> tuple[np.ndarray, int]:
    """Eq. combined_scheme applied ``nsteps`` times.  Returns (f, bad_ghosts)."""
    f = _f64(f)
    assert f.shape == (grid.nq, grid.nr, grid.nth)
    out = np.empty_like(f)
    g = grid.c()
    bad = lib().or_step(ctypes.byref(g), _p(f), _p(out), int(nsteps))
    return out, bad


def step_sample(grid: Grid, f: np.ndarray, nodes) -> np.ndarray:
    """One step of Eq. combined_scheme at the listed (i, j) nodes only;
    returns (len(nodes), 33).  ``f`` may be float32 or float64 (converted)."""
    f = _f64(f)
    assert f.shape == (grid.nq, grid.nr, grid.nth)
    nd = np.ascontiguousarray(np.asarray(nodes, dtype=np.int32).reshape(-1, 2))
    out = np.empty((len(nd), grid.nq))
    g = grid.c()
    lib().or_step_sample(ctypes.byref(g), _p(f), nd.ctypes.data_as(_I), len(nd), _p(out))
    return out


def init_feq(grid: Grid, rho, ur, ut, T) -> np.ndarray:
    rho, ur, ut, T = (_f64(a) for a in (rho, ur, ut, T))
    f = np.empty((grid.nq, grid.nr, grid.nth))
    g = grid.c()
    lib().or_init_feq(ctypes.byref(g), _p(rho), _p(ur), _p(ut), _p(T), _p(f))
    return f


def fields(grid: Grid, f: np.ndarray):
    """(rho, u_r, u_theta, T) of every node."""
    f = _f64(f)
    outs = [np.empty((grid.nr, grid.nth)) for _ in range(4)]
    g = grid.c()
    lib().or_fields(ctypes.byref(g), _p(f), *(_p(o) for o in outs))
    return tuple(outs)


def diagnostics(grid: Grid, f: np.ndarray) -> np.ndarray:
    """{mass, P_x, P_y, energy, min rho, min T, non-finite count, 0}."""
    f = _f64(f); out = np.zeros(8)
    g = grid.c()
    lib().or_diagnostics(ctypes.byref(g), _p(f), _p(out))
    return out


def adjoint_step(grid: Grid, f_t: np.ndarray, lam_next: np.ndarray,
                 tie_eps: float = TIE_FP64) -> np.ndarray:
    """lam_t = (dPhi/df at f_t)^T lam_next for one combined-scheme step, with
    the derivative convention of ``mwb_grad`` at the switch's kinks."""
    f_t = _f64(f_t); lam_next = _f64(lam_next)
    out = np.empty_like(f_t)
    g = grid.c()
    if lib().or_adjoint_step(ctypes.byref(g), _p(f_t), _p(lam_next), float(tie_eps), _p(out)):
        raise ValueError("the oracle's adjoint covers the combined MWB step only")
    return out


def adjoint_init(grid: Grid, rho, ur, ut, T, lam):
    """dJ/d(rho, u_r, u_theta, T) given lam = dJ/df at f = f^eq(fields)."""
    rho, ur, ut, T, lam = (_f64(a) for a in (rho, ur, ut, T, lam))
    outs = [np.empty((grid.nr, grid.nth)) for _ in range(4)]
    g = grid.c()
    lib().or_adjoint_init(ctypes.byref(g), _p(rho), _p(ur), _p(ut), _p(T), _p(lam),
                          *(_p(o) for o in outs))
    return tuple(outs)


#: names of the 12 polar components of each non-equilibrium kind
NONEQ_COMPONENTS = ("M2_rr", "M2_rt", "M2_tt", "M3_rrr", "M3_rrt", "M3_rtt", "M3_ttt",
                    "M31_r", "M31_t", "M42_rr", "M42_rt", "M42_tt")


def noneq(grid: Grid, f: np.ndarray) -> np.ndarray:
    """Sec. IV: (4, 12, nr, nth) array of M_m, M*_m, Delta_m, Delta*_m for
    m in {2, 3, (3,1), (4,2)}, polar components (NONEQ_COMPONENTS)."""
    f = _f64(f)
    out = np.empty((4, 12, grid.nr, grid.nth))
    g = grid.c()
    lib().or_noneq(ctypes.byref(g), _p(f), _p(out))
    return out


def noneq_sample(grid: Grid, f: np.ndarray, nodes) -> np.ndarray:
    """``noneq`` at the listed (i, j) nodes only: (len(nodes), 4, 12)."""
    f = _f64(f)
    nd = np.ascontiguousarray(np.asarray(nodes, dtype=np.int32).reshape(-1, 2))
    out = np.empty((len(nd), 4, 12))
    g = grid.c()
    lib().or_noneq_sample(ctypes.byref(g), _p(f), nd.ctypes.data_as(_I), len(nd), _p(out))
    return out


def num_threads() -> int:
    return lib().or_num_threads()


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))
