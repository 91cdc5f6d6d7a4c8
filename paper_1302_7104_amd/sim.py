"""Python front end of the HIP library: a simulation context whose state lives
in torch-owned device memory, and autograd Functions whose backward runs the
hand-written adjoint kernels with checkpoint-recompute.

PyTorch provides device memory and the stream; every step, moment, diagnostic
and adjoint computation runs in libpclb.so.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _native as N

NQ = 33   # velocities of the octagon; the double and triple octagon have 65 and 97


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Sim:
    """One annulus, one precision, one device.

    ``problem`` is any object with nr, nth, r1, r2, tau, dt, bc_kind, bc_par
    and optionally nf and ni (e.g. a ``workloads.Problem``; ni = 8, 16 or 24
    directions per speed, the state then holds 1 + 4 ni velocity planes).  ``strip_*`` set the
    launch shape of the strip kernel (0: default), ``adjoint_tie`` the tie
    threshold of the adjoint (0: the precision's default), ``scheme`` and
    ``relaxation`` the convection scheme and the relaxation form (the
    paper's combined scheme by default)."""

    def __init__(self, problem, precision: int = 32, kernel: int = N.KERNEL_AUTO,
                 device: str | torch.device = "cuda:0", strip_chunk: int = 0,
                 strip_order: int = N.ORDER_DEFAULT, adjoint_tie: float = 0.0,
                 scheme: int = N.SCHEME_MWB, relaxation: int = N.RELAX_ANALYTIC):
        if precision not in (32, 64):
            raise ValueError("precision must be 32 or 64")
        self.L = N.lib()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise RuntimeError("the HIP path needs a GPU device")
        torch.cuda.set_device(self.device)
        self.problem = problem
        self.precision = precision
        self.dtype = torch.float32 if precision == 32 else torch.float64
        self.nr, self.nth = problem.nr, problem.nth
        self.ni = int(getattr(problem, "ni", 8))
        self.nq = 1 + 4 * self.ni
        self.cfg = N.Config(problem.nr, problem.nth, problem.r1, problem.r2, problem.tau,
                            problem.dt, self.ni, getattr(problem, "nf", 8), precision, 1, kernel,
                            strip_chunk, strip_order, adjoint_tie, scheme, relaxation)
        ctx = ctypes.c_void_p()
        N.check(self.L.pclb_create(ctypes.byref(self.cfg), ctypes.byref(ctx)), None)
        self.ctx = ctx
        shape = (self.nq, self.nr, self.nth)
        self.buf = [torch.empty(shape, dtype=self.dtype, device=self.device),
                    torch.empty(shape, dtype=self.dtype, device=self.device)]
        self.stream = torch.cuda.current_stream(self.device)
        N.check(self.L.pclb_bind(self.ctx, _ptr(self.buf[0]), _ptr(self.buf[1]),
                                 ctypes.c_void_p(self.stream.cuda_stream)), self.ctx)
        for side in range(2):
            self.set_bc(side, problem.bc_kind[side], problem.bc_par[side])

    # -- lifetime --------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None):
            torch.cuda.synchronize(self.device)
            self.L.pclb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- configuration ---------------------------------------------------
    def set_bc(self, side: int, kind: int, params=(0.0, 0.0, 0.0, 0.0)):
        p = (ctypes.c_double * 4)(*[float(x) for x in (list(params) + [0.0] * 4)[:4]])
        N.check(self.L.pclb_set_bc(self.ctx, int(side), int(kind), p), self.ctx)

    def cfl_dt(self, cfl: float = 0.3) -> float:
        return self.L.pclb_cfl_dt(ctypes.byref(self.cfg), float(cfl))

    # -- state -------------------------------------------------------------
    def _field(self, a) -> torch.Tensor:
        t = torch.as_tensor(a, dtype=torch.float64, device=self.device)
        assert t.shape == (self.nr, self.nth), t.shape
        return t.contiguous()

    def init_state(self, rho, ur, ut, T):
        """f = f^eq(rho, u, T) on every node; fields in polar components."""
        fs = [self._field(a) for a in (rho, ur, ut, T)]
        N.check(self.L.pclb_init_state(self.ctx, *(_ptr(t) for t in fs)), self.ctx)

    @property
    def current(self) -> int:
        w = ctypes.c_int32()
        N.check(self.L.pclb_current(self.ctx, ctypes.byref(w)), self.ctx)
        return w.value

    @property
    def state(self) -> torch.Tensor:
        """The buffer holding the current f (a view of library-bound memory)."""
        return self.buf[self.current]

    def load_state(self, f: torch.Tensor):
        """Copy an arbitrary distribution into the current buffer."""
        self.state.copy_(f)

    @property
    def steps(self) -> int:
        s = ctypes.c_int64()
        N.check(self.L.pclb_step_count(self.ctx, ctypes.byref(s)), self.ctx)
        return s.value

    def step(self, n: int = 1):
        N.check(self.L.pclb_step(self.ctx, int(n)), self.ctx)

    def step_graph(self, n: int):
        """n steps as one replay of a captured HIP graph (same result as
        step(n)); worth it where kernel launches dominate a step."""
        N.check(self.L.pclb_step_graph(self.ctx, int(n)), self.ctx)

    def step_into(self, f_in: torch.Tensor, f_out: torch.Tensor):
        self._check_state_tensor(f_in)
        self._check_state_tensor(f_out)
        N.check(self.L.pclb_step_into(self.ctx, _ptr(f_in), _ptr(f_out)), self.ctx)

    def _check_state_tensor(self, t: torch.Tensor):
        if t.dtype != self.dtype or t.shape != (self.nq, self.nr, self.nth) or not t.is_contiguous() \
                or t.device != self.device:
            raise ValueError(f"state tensors must be contiguous ({self.nq}, nr, nth) of the context dtype")

    # -- diagnostics -------------------------------------------------------
    def fields(self, f: torch.Tensor | None = None):
        out = [torch.empty((self.nr, self.nth), dtype=torch.float64, device=self.device) for _ in range(4)]
        if f is None:
            N.check(self.L.pclb_moments(self.ctx, *(_ptr(o) for o in out), None), self.ctx)
        else:
            self._check_state_tensor(f)
            N.check(self.L.pclb_moments_of(self.ctx, _ptr(f), *(_ptr(o) for o in out), None), self.ctx)
        return dict(zip(("rho", "ur", "ut", "T"), out))

    def diagnostics(self, f: torch.Tensor | None = None) -> torch.Tensor:
        """Device tensor {mass, P_x, P_y, energy, min rho, min T, non-finite, step}."""
        d = torch.empty(8, dtype=torch.float64, device=self.device)
        if f is None:
            N.check(self.L.pclb_moments(self.ctx, None, None, None, None, _ptr(d)), self.ctx)
        else:
            self._check_state_tensor(f)
            N.check(self.L.pclb_moments_of(self.ctx, _ptr(f), None, None, None, None, _ptr(d)), self.ctx)
        return d

    def diagnostics_host(self) -> np.ndarray:
        out = (ctypes.c_double * 8)()
        N.check(self.L.pclb_moments_host(self.ctx, out), self.ctx)
        return np.array(out[:])

    def noneq(self, kinds: int = N.NONEQ_ALL, f: torch.Tensor | None = None) -> torch.Tensor:
        """Non-equilibrium fields (Sec. IV) of f (default: the current state):
        tensor (n_kinds, 12, nr, nth) of the selected kinds in the order M, M*,
        Delta, Delta*, 12 polar components each."""
        n = bin(int(kinds) & N.NONEQ_ALL).count("1")
        out = torch.empty((max(n, 1), 12, self.nr, self.nth), dtype=torch.float64, device=self.device)
        if f is not None:
            self._check_state_tensor(f)
        N.check(self.L.pclb_noneq(self.ctx, _ptr(f), int(kinds), _ptr(out)), self.ctx)
        return out

    # -- adjoint -----------------------------------------------------------
    def adjoint_step(self, f_t: torch.Tensor, lam_next: torch.Tensor, lam_out: torch.Tensor):
        for t in (f_t, lam_next, lam_out):
            self._check_state_tensor(t)
        N.check(self.L.pclb_adjoint_step(self.ctx, _ptr(f_t), _ptr(lam_next), _ptr(lam_out)), self.ctx)

    def adjoint_init(self, lam0: torch.Tensor, rho, ur, ut, T):
        self._check_state_tensor(lam0)
        fs = [self._field(a) for a in (rho, ur, ut, T)]
        outs = [torch.empty_like(fs[0]) for _ in range(4)]
        N.check(self.L.pclb_adjoint_init(self.ctx, _ptr(lam0), *(_ptr(t) for t in fs),
                                         *(_ptr(o) for o in outs)), self.ctx)
        return outs


# ---------------------------------------------------------------------------
# Autograd

class InitState(torch.autograd.Function):
    """(rho, u_r, u_theta, T) -> f^eq, with the adjoint-init kernel as backward."""

    @staticmethod
    def forward(ctx, sim: Sim, rho, ur, ut, T):
        sim.init_state(rho.detach(), ur.detach(), ut.detach(), T.detach())
        ctx.sim = sim
        ctx.save_for_backward(rho, ur, ut, T)
        return sim.state.clone()

    @staticmethod
    def backward(ctx, grad_f):
        sim = ctx.sim
        rho, ur, ut, T = ctx.saved_tensors
        g = grad_f.to(sim.dtype).contiguous()
        d = sim.adjoint_init(g, rho.detach(), ur.detach(), ut.detach(), T.detach())
        return (None, *d)


class Evolve(torch.autograd.Function):
    """f_0 -> f_n by n combined-scheme steps.  Backward: checkpoint every
    ``ckpt`` steps in the forward; per segment, recompute and store the
    segment's states, then run the adjoint step backwards through them.
    ``ckpt = 0`` keeps every state of the forward in device memory instead
    ((n + 1) states: 55 GB for 200 FP32 steps on 1024 x 2048), so that the
    backward pass runs the adjoint steps alone, without recompute."""

    @staticmethod
    def forward(ctx, sim: Sim, f0: torch.Tensor, n: int, ckpt: int = 20):
        if ckpt < 0:
            raise ValueError("ckpt must be >= 0 (0: keep every state)")
        if ckpt == 0:
            need = (n + 1) * sim.state.numel() * sim.state.element_size()
            free, _ = torch.cuda.mem_get_info(sim.device)
            if need > free:
                raise MemoryError(f"keeping {n + 1} states takes {need / 2**30:.1f} GiB, "
                                  f"{free / 2**30:.1f} GiB free: use ckpt > 0")
            traj = [f0.detach().to(sim.dtype).contiguous().clone()]
            for _ in range(n):
                nxt = torch.empty_like(traj[0])
                sim.step_into(traj[-1], nxt)
                traj.append(nxt)
            sim.load_state(traj[-1])
            ctx.sim, ctx.n, ctx.ckpt, ctx.ckpts, ctx.traj = sim, n, 0, None, traj
            return traj[-1].clone()
        sim.load_state(f0.detach())
        ckpts = []
        done = 0
        while done < n:
            ckpts.append(sim.state.clone())
            m = min(ckpt, n - done)
            sim.step(m)
            done += m
        ctx.sim, ctx.n, ctx.ckpt, ctx.ckpts, ctx.traj = sim, n, ckpt, ckpts, None
        return sim.state.clone()

    @staticmethod
    def backward(ctx, grad_fn):
        sim, n, ckpt = ctx.sim, ctx.n, ctx.ckpt
        lam = grad_fn.to(sim.dtype).contiguous().clone()
        lam_next = torch.empty_like(lam)
        if ctx.traj is not None:
            for t in reversed(range(n)):
                sim.adjoint_step(ctx.traj[t], lam, lam_next)
                lam, lam_next = lam_next, lam
            ctx.traj = None
            return None, lam, None, None
        seg_states = [torch.empty_like(lam) for _ in range(ckpt)]
        for s in reversed(range(len(ctx.ckpts))):
            start = s * ckpt
            m = min(ckpt, n - start)
            seg_states[0].copy_(ctx.ckpts[s])
            for t in range(1, m):
                sim.step_into(seg_states[t - 1], seg_states[t])
            for t in reversed(range(m)):
                sim.adjoint_step(seg_states[t], lam, lam_next)
                lam, lam_next = lam_next, lam
        ctx.ckpts = None
        return None, lam, None, None
