"""Material-interface tracking for the Richtmyer-Meshkov runs (Sec. III.C):
Lagrangian markers carried by the flow.  The model has one fluid; the two
media differ only in density, so the interface is followed as the set of
fluid particles that start on it.  Host-side post-processing of the fields
the GPU returns (no part of a step)."""
from __future__ import annotations

import numpy as np


def _interp(field, r, th, r1, dr, dth):
    """Bilinear interpolation of a node field [i, j] (r_i = r1 + i dr,
    theta_j = (j + 1) dth, periodic in theta over the grid's span; polar
    components repeat with the domain) at points (r, th)."""
    nr, nth = field.shape
    x = (r - r1) / dr
    y = th / dth - 1.0
    i0 = np.clip(np.floor(x).astype(int), 0, nr - 2)
    fx = np.clip(x - i0, 0.0, 1.0)
    j0 = np.floor(y).astype(int)
    fy = y - j0
    j0 %= nth
    j1 = (j0 + 1) % nth
    f00, f01 = field[i0, j0], field[i0, j1]
    f10, f11 = field[i0 + 1, j0], field[i0 + 1, j1]
    return (1 - fx) * ((1 - fy) * f00 + fy * f01) + fx * ((1 - fy) * f10 + fy * f11)


def track_amplitude(sim, problem, markers: int = 450, every: int = 20, t_end: float = 0.2):
    """Advance `sim` (already initialised) to t_end, carrying markers that
    start on r = R + A0 cos(k R theta) with the flow velocity (Heun's rule
    over every `every` steps).  Returns arrays (t, amplitude, signed
    amplitude, mean radius): the amplitude is half the largest radial
    distance between markers (crest to trough, as the paper defines it), the
    signed one the markers' cos(k R theta_0) component (negative once the
    interface has inverted)."""
    p = problem.params
    span = 2.0 * np.pi * problem.nf / 8.0
    th = (np.arange(markers) + 0.5) * span / markers
    r = p["R"] + p["A0"] * np.cos(p["k"] * p["R"] * th)
    r1, dr, dth = problem.r1, problem.dr, problem.dth

    def vel(fl, rr, tt):
        ur = _interp(fl[0], rr, tt, r1, dr, dth)
        ut = _interp(fl[1], rr, tt, r1, dr, dth)
        return ur, ut / rr

    def fields():
        f = sim.fields()
        return f["ur"].cpu().numpy(), f["ut"].cpu().numpy()

    h = every * problem.dt
    n = int(round(t_end / h))
    mode = np.cos(p["k"] * p["R"] * th)

    def signed(rr):
        return 2.0 * np.mean((rr - rr.mean()) * mode)

    ts, amp, sgn, mean = [0.0], [0.5 * (r.max() - r.min())], [signed(r)], [r.mean()]
    cur = fields()
    for s in range(n):
        a_r, a_t = vel(cur, r, th)
        sim.step(every)
        nxt = fields()
        rp, tp = r + h * a_r, th + h * a_t
        b_r, b_t = vel(nxt, rp, tp)
        r = r + 0.5 * h * (a_r + b_r)
        th = th + 0.5 * h * (a_t + b_t)
        cur = nxt
        ts.append((s + 1) * h)
        amp.append(0.5 * (r.max() - r.min()))
        sgn.append(signed(r))
        mean.append(r.mean())
    return np.array(ts), np.array(amp), np.array(sgn), np.array(mean)


def compression(t, amp, signed, A0, R, shock_r, shock_speed, t_comp=0.03):
    """The quantities the paper reads off its Figs. 8 and 10, with time zero
    where the incident shock reaches the interface's trough:
      ratio      the amplitude t_comp = 0.03 later (the paper's end of the
                 compression stage in both runs) over A0: the compression ratio;
      A_min, t_min  the smallest amplitude in the first 0.1 and its time;
      t_zero     the first time the signed amplitude changes sign (the
                 interface inverts; heavy to light), or None;
      t_reco     the first time after t_min and t_zero at which the amplitude
                 is back at A0, or None within the run."""
    t0 = (R - A0 - shock_r) / shock_speed
    a_tc = float(np.interp(t0 + t_comp, t, amp))
    sel = (t >= t0) & (t <= t0 + 0.1)
    k = int(np.argmin(np.where(sel, amp, np.inf)))
    flips = np.nonzero((t > t0) & (np.sign(signed) != np.sign(signed[0])))[0]
    t_zero = None
    if len(flips):
        m = flips[0]
        # linear interpolation of the crossing between the last two samples
        t_zero = float(t[m - 1] + (t[m] - t[m - 1]) * signed[m - 1] / (signed[m - 1] - signed[m]) - t0)
    start = max(t[k], t0 + (t_zero if t_zero is not None else 0.0))
    after = np.nonzero((t > start) & (amp >= A0))[0]
    return {"t_meet": t0, "A_at_t_comp": a_tc, "ratio": a_tc / A0,
            "A_min": float(amp[k]), "t_min": float(t[k] - t0), "t_zero": t_zero,
            "t_reco": float(t[after[0]] - t0) if len(after) else None}
