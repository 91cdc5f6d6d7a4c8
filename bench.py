#!/usr/bin/env python3
"""Throughput of the polar FDLB combined-scheme step on one MI355X.

Workload (the headline configuration): Kelvin-Helmholtz shear layer on the
annulus r in [0.5, 1.5] with 4096 x 8192 nodes and 33 velocities, FP32 state,
tau = 1e-5, Courant number 0.25 (the recipe's: the combined scheme is
unstable next to the inner wall at 0.3); W warm-up steps, then K timed steps.
One step = one pass of the whole hot path (radial ghost layers, moments,
equilibrium, relaxation, MWB convection in r and theta, store) over the whole
grid.  The time per step does not depend on the Courant number.

Printed: one JSON line with the metric (G cell-velocity updates per second),
the roofline of the step kernel (algorithmic bytes / kernel time vs 8 TB/s),
the CPU oracle timed on this host on a bounded sample, and extra figures: the
FP64 step on the same grid, the adjoint/forward cost ratio on the
1024 x 2048 Richtmyer-Meshkov adjoint configuration, and the FP32 error
against FP64 after the full run of every configuration.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
NQ = 33


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("common.h", "strip_common.h", "k_strip.hip", "k_forward.hip"):
        with open(os.path.join(ROOT, "paper_1302_7104_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(precision: int, nodes: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    entry = rec.get(f"fp{precision}")
    if not entry or entry.get("nodes") != nodes:
        return None
    return entry.get("bytes_per_launch")


def time_steps(sim, torch, steps: int) -> float:
    """Average ms per step over `steps` steps, HIP events on the sim's stream."""
    st = sim.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    sim.step(steps)
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def run_forward(W, Sim, torch, precision, steps, warmup, nr=4096, nth=8192):
    P, F = W.kelvin_helmholtz(nr, nth, steps)
    sim = Sim(P, precision=precision)
    sim.init_state(F["rho"], F["ur"], F["ut"], F["T"])
    del F
    sim.step(warmup)
    ms = time_steps(sim, torch, steps)
    d = sim.diagnostics_host()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return P, ms, d


def run_variants(W, Sim, torch, steps=20, warmup=3):
    """FP32 step time on the headline workload for each convection scheme and
    relaxation form (MWB and the two upwind comparison schemes on the strip
    kernel, Lax-Wendroff on the node kernel, MWB also on the node kernel for
    reference), and the time of the non-equilibrium fields kernel (all four
    kinds) on the same state."""
    import ctypes
    from paper_1302_7104_amd import _native as N
    P, F = W.kelvin_helmholtz(4096, 8192, steps)
    nodes = P.nr * P.nth
    step_bytes = 2 * NQ * nodes * 4
    out = {}
    variants = (("mwb_strip", {}), ("mwb_node", {"kernel": N.KERNEL_NODE}),
                ("mwb_euler_relaxation_strip", {"relaxation": N.RELAX_EULER}),
                ("warming_beam_strip", {"scheme": N.SCHEME_WB}),
                ("lax_wendroff_node", {"scheme": N.SCHEME_LW}),
                ("upwind2_strip", {"scheme": N.SCHEME_UPWIND2}))
    for name, kw in variants:
        sim = Sim(P, precision=32, **kw)
        sim.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        sim.step(warmup)
        ms = time_steps(sim, torch, steps)
        out[name] = {"ms_per_step": ms, "hbm_frac": step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        if name == "mwb_strip":
            # Sec. IV fields: read the state (132 B per node), write 4 kinds x 12
            # components in double (384 B per node)
            res = torch.empty((4, 12, P.nr, P.nth), dtype=torch.float64, device=sim.device)
            ptr = ctypes.c_void_p(res.data_ptr())
            N.check(sim.L.pclb_noneq(sim.ctx, None, N.NONEQ_ALL, ptr), sim.ctx)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(sim.stream)
            for _ in range(5):
                N.check(sim.L.pclb_noneq(sim.ctx, None, N.NONEQ_ALL, ptr), sim.ctx)
            e1.record(sim.stream)
            torch.cuda.synchronize()
            ms_nq = e0.elapsed_time(e1) / 5
            nq_bytes = nodes * (NQ * 4 + 4 * 12 * 8)
            out["noneq_all_kinds"] = {"ms": ms_nq, "bytes_per_node": NQ * 4 + 4 * 12 * 8,
                                      "achieved_gbs": nq_bytes / (ms_nq * 1e-3) / 1e9,
                                      "hbm_frac": nq_bytes / (ms_nq * 1e-3) / 1e9 / HBM_PEAK_GBS}
            del res
        sim.close()
        del sim
        torch.cuda.empty_cache()
    return out


def run_models(W, Sim, torch, steps=20, warmup=3):
    """Step time of the double and triple octagon (Table I rows 2 and 3: 65
    and 97 velocities) on the headline workload's grid, both precisions.
    Algorithmic bytes per step: each velocity value read once and written
    once."""
    import dataclasses
    P0, F = W.kelvin_helmholtz(4096, 8192, steps)
    nodes = P0.nr * P0.nth
    out = {}
    for ni in (16, 24):
        P = dataclasses.replace(P0, ni=ni, nf=ni)
        nq = 1 + 4 * ni
        for prec in (32, 64):
            sim = Sim(P, precision=prec)
            sim.init_state(F["rho"], F["ur"], F["ut"], F["T"])
            sim.step(warmup)
            ms = time_steps(sim, torch, steps)
            d = sim.diagnostics_host()
            sim.close()
            del sim
            torch.cuda.empty_cache()
            byts = 2 * nq * nodes * (prec // 8)
            out[f"ni{ni}_fp{prec}"] = {
                "velocities": nq, "ms_per_step": ms,
                "gcellvel_per_s": nq * nodes / (ms * 1e-3) / 1e9,
                "hbm_frac": byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "finite": bool(d[6] == 0)}
    return out


def graph_replay_rotation(W, Sim, torch, steps=200, reps=5):
    """The rotation configuration (64 x 128, 200 steps): per-step time of
    eager launches (pclb_step) against one replayed HIP graph of the 200
    steps (pclb_step_graph), FP32; the grid is small enough for launches to
    dominate."""
    P, F = W.rotation(64, 128, steps)
    out = {}
    for name in ("eager", "graph"):
        sim = Sim(P, precision=32)
        sim.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        run = sim.step if name == "eager" else sim.step_graph
        run(steps)                          # warm-up (and the capture)
        st = sim.stream
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(st)
        for _ in range(reps):
            run(steps)
        e1.record(st)
        torch.cuda.synchronize()
        out[f"{name}_us_per_step"] = e0.elapsed_time(e1) * 1e3 / (reps * steps)
        sim.close()
    return out


def couette_errors(W, Sim, torch):
    """Sec. III.A: the one-eighth-sector rotating-cylinder run (100 x 20) from
    rest to steady state in FP64 for each relaxation time; the largest
    departure of the theta-mean u_theta from Eq. RSF, relative to R2 omega2."""
    import numpy as np
    out = {}
    for tau, t_end in ((0.2, 10.0), (0.1, 15.0), (0.05, 20.0), (0.01, 40.0)):
        P, F = W.couette(tau=tau, steps=int(round(t_end / 1e-3)))
        sim = Sim(P, precision=64)
        sim.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        sim.step(P.steps)
        u = sim.fields()["ut"].mean(1).cpu().numpy()
        sim.close()
        R, _ = W.node_coords(P.nr, P.nth, P.r1, P.r2, P.nf)
        out[f"tau_{tau:g}"] = float(np.abs(u - W.couette_profile(R[:, 0])).max() / 0.2)
    return out


def rm_sector_runs(W, Sim):
    """Sec. III.C: the paper's two Richtmyer-Meshkov runs (1000 x 450, one
    eighth of the annulus, FP64) with the interface followed by markers;
    the compression ratio, the inversion and recovery times."""
    from paper_1302_7104_amd import interface as I
    out = {}
    for name, lth, t_end in (("light_to_heavy", True, 0.17), ("heavy_to_light", False, 0.32)):
        P, F = W.rm_sector(light_to_heavy=lth)
        sim = Sim(P, precision=64)
        sim.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        t, amp, sgn, _ = I.track_amplitude(sim, P, every=20, t_end=t_end)
        sim.close()
        p = P.params
        c = I.compression(t, amp, sgn, p["A0"], p["R"], p["shock_r"], p["shock_speed"])
        c["paper"] = {"ratio": 0.715, "theory": 0.758, "t_reco": 0.13} if lth else \
            {"ratio": 0.65, "theory": 0.61, "t_zero": 0.27, "t_reco": 0.66}
        out[name] = c
    return out


def adjoint_gradient(W, torch, Sim, Evolve, InitState, P, steps, ckpt, precision):
    """J = sum over 1.1 < r < 1.5 of rho^2 r dr dtheta after `steps` steps of
    the Richtmyer-Meshkov recipe, and dJ/da_k through the hand-written
    adjoint with checkpoint-recompute (ckpt = 0: every state kept).
    Returns (J, grad, forward ms/step, backward ms/step)."""
    sim = Sim(P, precision=precision)
    dev = sim.device
    amps = torch.as_tensor(W.rm_amplitudes(1), device=dev).requires_grad_(True)
    _, Ft = W.richtmyer_meshkov(P.nr, P.nth, steps, amps=amps, xp=torch)
    f0 = InitState.apply(sim, Ft["rho"], Ft["ur"], Ft["ut"], Ft["T"])
    torch.cuda.synchronize()
    sim.load_state(f0.detach())
    ms_fwd = time_steps(sim, torch, steps)
    R, _ = W.node_coords(P.nr, P.nth, P.r1, P.r2)
    band = torch.as_tensor(((R > 1.1) & (R < 1.5)) * R * P.dr * P.dth, device=dev,
                           dtype=sim.dtype)
    torch.cuda.synchronize()
    fn = Evolve.apply(sim, f0, steps, ckpt)
    J = ((fn.sum(0) ** 2) * band).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    grad = amps.grad.detach().cpu().numpy()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return float(J.item()), grad, ms_fwd, (t2 - t1) * 1e3 / steps


def fd_gradient(W, torch, Sim, P, steps, h):
    """Central differences of J in a_k with the FP64 forward."""
    import numpy as np
    sim = Sim(P, precision=64)
    R, _ = W.node_coords(P.nr, P.nth, P.r1, P.r2)
    band = torch.as_tensor(((R > 1.1) & (R < 1.5)) * R * P.dr * P.dth, device=sim.device)
    a0 = W.rm_amplitudes(1)

    def J_of(a):
        _, F = W.richtmyer_meshkov(P.nr, P.nth, steps, amps=a)
        sim.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        sim.step(steps)
        return float(((sim.state.sum(0) ** 2) * band).sum().item())

    fd = np.array([(J_of(a0 + h * np.eye(13)[k]) - J_of(a0 - h * np.eye(13)[k])) / (2 * h)
                   for k in range(13)])
    sim.close()
    return fd


def run_adjoint(W, torch, steps=200, ckpt=20):
    """The 1024 x 2048 Richtmyer-Meshkov adjoint configuration: cost of the
    FP32 backward pass relative to the FP32 forward step, the FP32 and FP64
    gradients, and their agreement with FP64 central differences."""
    import numpy as np
    from paper_1302_7104_amd.sim import Evolve, InitState, Sim
    P, _ = W.richtmyer_meshkov(1024, 2048, steps)
    J32, g32, fwd32, bwd32 = adjoint_gradient(W, torch, Sim, Evolve, InitState, P, steps, ckpt, 32)
    J64, g64, fwd64, bwd64 = adjoint_gradient(W, torch, Sim, Evolve, InitState, P, steps, ckpt, 64)
    # every state kept in HBM by the forward: the backward pass without recompute
    _, g32s, _, bwd32s = adjoint_gradient(W, torch, Sim, Evolve, InitState, P, steps, 0, 32)
    _, g64s, _, bwd64s = adjoint_gradient(W, torch, Sim, Evolve, InitState, P, steps, 0, 64)

    def rel(a, b):
        return float(np.abs(a - b).max() / np.abs(b).max())

    fd = {}
    for n, h in ((steps, 1e-4), (steps, 1e-6), (20, 1e-6)):
        P_n, _ = W.richtmyer_meshkov(1024, 2048, n)
        f = fd_gradient(W, torch, Sim, P_n, n, h)
        g_n = g64 if n == steps else adjoint_gradient(W, torch, Sim, Evolve, InitState, P_n, n,
                                                      ckpt, 64)[1]
        fd[f"{n}_steps_h{h:g}"] = {"fp64_adjoint_vs_fd": rel(g_n, f)}
        if n == steps:
            fd[f"{n}_steps_h{h:g}"]["fp32_adjoint_vs_fd"] = rel(g32, f)
    return dict(ms_forward_step=fwd32, ms_backward_per_step=bwd32,
                adjoint_over_forward=bwd32 / fwd32,
                fp64_ms_forward_step=fwd64, fp64_ms_backward_per_step=bwd64,
                fp64_adjoint_over_forward=bwd64 / fwd64,
                J_fp32=J32, J_fp64=J64, dJ_da_fp32=g32.tolist(), dJ_da_fp64=g64.tolist(),
                fp32_vs_fp64_gradient=rel(g32, g64), finite_differences=fd,
                stored_trajectory=dict(
                    ms_backward_per_step=bwd32s, adjoint_over_forward=bwd32s / fwd32,
                    fp64_ms_backward_per_step=bwd64s, fp64_adjoint_over_forward=bwd64s / fwd64,
                    same_gradients=bool(np.array_equal(g32s, g32) and np.array_equal(g64s, g64))))


def adjoint_kernel_times(W, torch, steps=50):
    """Adjoint step alone (ghost layers, ghost adjoint, node adjoint) against
    the forward step, on one state of the 1024 x 2048 Richtmyer-Meshkov
    recipe, with a seeded random cotangent; FP32 and FP64."""
    from paper_1302_7104_amd.sim import Sim
    res = {}
    gen = torch.Generator(device="cuda").manual_seed(0)
    for prec in (32, 64):
        P, F = W.richtmyer_meshkov(1024, 2048, 200)
        sim = Sim(P, precision=prec)
        sim.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        sim.step(5)
        f = sim.state.clone()
        lam = torch.randn(f.shape, generator=gen, device=f.device, dtype=f.dtype)
        out = torch.empty_like(f)
        for _ in range(5):
            sim.adjoint_step(f, lam, out)
        st = sim.stream
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(st)
        for _ in range(steps):
            sim.adjoint_step(f, lam, out)
        e1.record(st)
        torch.cuda.synchronize()
        ta = e0.elapsed_time(e1) / steps
        tf = time_steps(sim, torch, steps)
        res[f"fp{prec}"] = {"adjoint_step_ms": ta, "forward_step_ms": tf, "ratio": ta / tf}
        sim.close()
        del sim
        torch.cuda.empty_cache()
    return res


#: the configurations run to their full length for the FP32 error statement:
#: name -> (recipe, n_r, n_theta, steps)
ACCURACY_RUNS = {
    "rotation_64x128": ("rotation", 64, 128, 200),
    "shock_tube_512x1024": ("shock_tube", 512, 1024, 2000),
    "richtmyer_meshkov_2048x4096": ("richtmyer_meshkov", 2048, 4096, 5000),
    "kelvin_helmholtz_4096x8192": ("kelvin_helmholtz", 4096, 8192, 1050),
    "adjoint_rm_1024x2048": ("richtmyer_meshkov", 1024, 2048, 200),
}


def smooth_mask(torch, rho, jump=0.01, width=2):
    """Nodes whose (2 width + 1)^2 neighbourhood (theta periodic, r clamped)
    holds no relative density jump above `jump`: (max - min) / rho < jump."""
    hi = rho.clone()
    lo = rho.clone()
    nr = rho.shape[0]
    for di in range(-width, width + 1):
        rows = torch.clamp(torch.arange(nr, device=rho.device) + di, 0, nr - 1)
        shifted = rho[rows]
        for dj in range(-width, width + 1):
            x = torch.roll(shifted, -dj, dims=1)
            hi = torch.maximum(hi, x)
            lo = torch.minimum(lo, x)
    return (hi - lo) / rho < jump


def moment_errors(torch, fa, fb, mask):
    """Largest relative errors of field set fa against the reference fb over
    the masked nodes: rho and T relative, the velocity relative to the local
    sound speed sqrt(2 T) (gamma = 2)."""
    rho, T = fb["rho"], fb["T"]
    c = torch.sqrt(2.0 * T)
    du = torch.sqrt((fa["ur"] - fb["ur"]) ** 2 + (fa["ut"] - fb["ut"]) ** 2) / c
    out = {}
    for key, err in (("rho", (fa["rho"] - rho).abs() / rho), ("T", (fa["T"] - T).abs() / T),
                     ("u_over_c", du)):
        out[key] = float(err[mask].max().item()) if bool(mask.any()) else 0.0
        out[key + "_all_nodes"] = float(err.max().item())
    return out


def fp32_accuracy(W, torch, name):
    """FP32 against FP64 after the full run of one configuration: both
    precisions through the HIP path from the same fields (the FP64 path is
    the one the parity tests hold to the oracle).  Returns the smooth-region
    errors of rho, T and u, the share of nodes in the smooth region, the
    largest errors over all nodes, and the same errors for an FP64 run started
    from the initial state rounded to float (how much the flow itself
    amplifies a perturbation of the size of float rounding)."""
    from paper_1302_7104_amd.sim import Sim
    recipe, nr, nth, steps = ACCURACY_RUNS[name]
    P, F = getattr(W, recipe)(nr=nr, nth=nth, steps=steps)
    fields = {}
    for key, prec in (("fp64", 64), ("fp32", 32), ("fp64_rounded_start", 64)):
        sim = Sim(P, precision=prec)
        sim.init_state(F["rho"], F["ur"], F["ut"], F["T"])
        if key == "fp64_rounded_start":
            sim.state.copy_(sim.state.float().double())
        sim.step(steps)
        fields["diag_" + key] = sim.diagnostics_host()
        fields[key] = sim.fields()
        sim.close()
        del sim
        torch.cuda.empty_cache()
    mask = smooth_mask(torch, fields["fp64"]["rho"])
    res = moment_errors(torch, fields["fp32"], fields["fp64"], mask)
    res["steps"] = steps
    res["cfl"] = W.CFL[recipe]
    res["smooth_fraction"] = float(mask.double().mean().item())
    d32, d64 = fields["diag_fp32"], fields["diag_fp64"]
    res["mass_rel_fp32_vs_fp64"] = abs(d32[0] - d64[0]) / d64[0]
    res["fp64_rounded_start"] = moment_errors(torch, fields["fp64_rounded_start"], fields["fp64"], mask)
    del fields
    torch.cuda.empty_cache()
    return res


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W, target_s=20.0, one_thread_s=5.0):
    """The FP64 CPU oracle, as it stands, on the same recipe at 512 x 1024
    (cost per cell-velocity update does not depend on the grid size), on all
    the host threads OpenMP offers and on one thread."""
    from oracle import oracle as O
    O.build(force=False)
    P, F = W.kelvin_helmholtz(512, 1024, 1)
    g = O.Grid(P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, P.bc_kind, P.bc_par, nf=P.nf)
    f = O.init_feq(g, **F)

    def rate(budget):
        nonlocal f
        f, _ = O.step(g, f, 1)                   # thread pool start-up
        t0 = time.perf_counter()
        f, _ = O.step(g, f, 1)
        one = time.perf_counter() - t0
        n = max(1, int(budget / max(one, 1e-3)))
        t0 = time.perf_counter()
        f, _ = O.step(g, f, n)
        dt = time.perf_counter() - t0
        return NQ * P.nr * P.nth * n / dt / 1e9, n, dt

    threads = O.num_threads()
    r_all, n_all, t_all = rate(target_s)
    O.set_threads(1)
    r_one, n_one, t_one = rate(one_thread_s)
    O.set_threads(threads)
    return {"value": r_all, "unit": "Gcell\u00b7vel/s", "cores": threads, "kind": "oracle",
            "one_thread_value": r_one, "cpu": cpu_model(),
            "sample": f"kelvin_helmholtz recipe at 512x1024 (33 velocities): {n_all} FP64 steps "
                      f"in {t_all:.1f} s on {threads} OpenMP threads, {n_one} steps in "
                      f"{t_one:.1f} s on one thread"}


def calibrate_copy(torch, gib=1):
    """A plain device-to-device copy of `gib` GiB, three times: the reference
    that scales the FETCH_SIZE / WRITE_SIZE counters to bytes."""
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()


def _counter_values(csv_path, counter):
    """Per-dispatch values of one rocprofv3 counter, listed per kernel name."""
    import csv
    from collections import defaultdict
    per = defaultdict(float)
    names = {}
    with open(csv_path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            per[r["Dispatch_Id"]] += float(r["Counter_Value"])
            names[r["Dispatch_Id"]] = r["Kernel_Name"]
    agg = defaultdict(list)
    for d, v in per.items():
        agg[names[d]].append(v)
    return agg


def summarize_counters(fetch_csv, write_csv, nodes, precision=32, copy_gib=1):
    """Turn the two counter passes into HBM bytes per step-kernel launch.
    Each counter is scaled by what it reads for the plain copy of known size
    (copy bytes / counter value), then stored with the kernel source hash."""
    fetch = _counter_values(fetch_csv, "FETCH_SIZE")
    write = _counter_values(write_csv, "WRITE_SIZE")
    copy_bytes = copy_gib * (1 << 30)

    def vals(d, key):
        return [v for k, vs in d.items() if key in k for v in vs]

    # the copy of known size is the largest copy dispatch; a step launches the
    # ghost kernel once and the strip kernel twice (uniform strips, then the
    # others): bytes per step = all strip-kernel dispatches / ghost dispatches
    f_copy, w_copy = max(vals(fetch, "copyBuffer")), max(vals(write, "copyBuffer"))
    n_steps = len(vals(fetch, "ghost_kernel"))
    assert n_steps == len(vals(write, "ghost_kernel")) and n_steps > 0
    f_step = sum(vals(fetch, "step_strip_kernel")) / n_steps
    w_step = sum(vals(write, "step_strip_kernel")) / n_steps
    f_scale, w_scale = copy_bytes / f_copy, copy_bytes / w_copy
    rec = {"source_hash": kernel_source_hash(),
           f"fp{precision}": {"nodes": nodes, "fetch_bytes": f_step * f_scale,
                              "write_bytes": w_step * w_scale,
                              "bytes_per_launch": f_step * f_scale + w_step * w_scale,
                              "fetch_counter_per_copy_byte": f_copy / copy_bytes,
                              "write_counter_per_copy_byte": w_copy / copy_bytes,
                              "algorithmic_bytes": 2 * NQ * nodes * (precision // 8)}}
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--fp64-steps", type=int, default=200)
    ap.add_argument("--no-extras", action="store_true", help="headline FP32 step only")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--fp64-only", action="store_true",
                    help="time the FP64 step (node kernel) on the same workload and exit")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="time the adjoint step alone against the forward step (1024 x 2048 "
                         "Richtmyer-Meshkov) and exit")
    ap.add_argument("--accuracy-only", action="store_true",
                    help="FP32 error against FP64 after the full run of every configuration")
    ap.add_argument("--variants-only", action="store_true",
                    help="step time per convection scheme, the non-equilibrium fields kernel, "
                         "the Couette errors and the sector Richtmyer-Meshkov runs, then exit")
    ap.add_argument("--models-only", action="store_true",
                    help="time the double and triple octagon (65 and 97 velocities) on the "
                         "headline grid and exit")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/step_kernel_traffic.json from two rocprofv3 --pmc "
                         "runs (FETCH_SIZE, WRITE_SIZE) of this script and exit")
    args = ap.parse_args()
    if args.summarize_counters:
        rec = summarize_counters(*args.summarize_counters, nodes=4096 * 8192)
        with open(os.path.join(ROOT, "profiles", "step_kernel_traffic.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU execution "
                          "(theta-sector sharding with halo exchange) is not built", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_1302_7104_amd import workloads as W
    from paper_1302_7104_amd.sim import Sim

    if args.fp64_only:
        P64, ms64, _ = run_forward(W, Sim, torch, 64, args.steps, args.warmup)
        nodes = P64.nr * P64.nth
        print(json.dumps({"workload": "kelvin_helmholtz_4096x8192", "precision": 64,
                          "ms_per_step": ms64,
                          "gcellvel_per_s": NQ * nodes / (ms64 * 1e-3) / 1e9,
                          "hbm_frac": 2 * NQ * nodes * 8 / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS}),
              flush=True)
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint_rm_1024x2048": adjoint_kernel_times(W, torch)}), flush=True)
        return
    if args.accuracy_only:
        for name in ACCURACY_RUNS:
            print(json.dumps({name: fp32_accuracy(W, torch, name)}), flush=True)
        return
    if args.models_only:
        print(json.dumps({"double_triple_octagon_kh4096x8192": run_models(W, Sim, torch),
                          "rotation_64x128_graph_replay": graph_replay_rotation(W, Sim, torch)}),
              flush=True)
        return
    if args.variants_only:
        print(json.dumps({"schemes_and_noneq_kh4096x8192_fp32": run_variants(W, Sim, torch)}),
              flush=True)
        print(json.dumps({"couette_sector_steady_error": couette_errors(W, Sim, torch)}), flush=True)
        print(json.dumps({"rm_sector_compression": rm_sector_runs(W, Sim)}), flush=True)
        return
    P, ms, diag = run_forward(W, Sim, torch, 32, args.steps, args.warmup)
    if args.calibrate_copy:
        calibrate_copy(torch)
    nodes = P.nr * P.nth
    cellvel = NQ * nodes
    value = cellvel / (ms * 1e-3) / 1e9
    bytes_launch = 2 * NQ * nodes * 4
    achieved = bytes_launch / (ms * 1e-3) / 1e9
    traffic = stored_traffic(32, nodes)
    out = {
        "metric": "Gcell\u00b7vel updates/s + HBM GB/s %peak, FP32 vs FP64 step; adjoint/fwd cost",
        "value": value,
        "unit": "Gcell\u00b7vel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "kelvin_helmholtz_4096x8192", "n_r": P.nr, "n_theta": P.nth,
                   "velocities": NQ, "precision": "fp32 state, fp64 collision", "dt": P.dt,
                   "tau": P.tau, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
    }
    extra = {"mass_after_run": diag[0], "min_rho": diag[4], "min_T": diag[5]}
    if not args.no_extras:
        P64, ms64, _ = run_forward(W, Sim, torch, 64, args.fp64_steps, 10)
        extra["fp64_ms_per_step"] = ms64
        extra["fp64_gcellvel_per_s"] = cellvel / (ms64 * 1e-3) / 1e9
        extra["fp64_hbm_frac"] = (2 * NQ * nodes * 8) / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS
        extra["adjoint_rm_1024x2048"] = run_adjoint(W, torch)
        extra["fp32_error_vs_fp64_after_run"] = {name: fp32_accuracy(W, torch, name)
                                                 for name in ACCURACY_RUNS}
        extra["schemes_and_noneq_kh4096x8192_fp32"] = run_variants(W, Sim, torch)
        extra["double_triple_octagon_kh4096x8192"] = run_models(W, Sim, torch)
        extra["rotation_64x128_graph_replay"] = graph_replay_rotation(W, Sim, torch)
        extra["couette_sector_steady_error"] = couette_errors(W, Sim, torch)
        extra["rm_sector_compression"] = rm_sector_runs(W, Sim)
    out["extra"] = extra
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
