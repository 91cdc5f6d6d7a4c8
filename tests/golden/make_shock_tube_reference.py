"""Writes tests/golden/shock_tube_512x1024_oracle.npz: the FP64 oracle's state
of the shock-tube recipe (512 x 1024, its full 2000 steps) reduced to what the
GPU parity test compares:

* radial profiles of rho, u_r, u_theta and T after the run (mean, minimum and
  maximum over theta), the comparison the recipe itself names;
* all 33 distributions at 400 seeded sample nodes (every row next to a wall,
  the rest at random);
* the same samples from a second oracle run that is perturbed by 32 ulps of
  random noise after every step: their distance from the first run is the
  amplification of rounding differences that the problem itself shows;
* the conserved totals of the final state.

Calls only the oracle and the input generator.  Run from the repository root:
    python tests/golden/make_shock_tube_reference.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1302_7104_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "shock_tube_512x1024_oracle.npz")
NOISE_ULPS = 32


def sample_nodes(nr, nth, n, seed):
    rng = np.random.default_rng(seed)
    walls = [(i, j) for i in (0, 1, 2, nr - 3, nr - 2, nr - 1) for j in (0, 1, nth // 2, nth - 1)]
    rand = [(int(a), int(b)) for a, b in zip(rng.integers(0, nr, n), rng.integers(0, nth, n))]
    return np.array(walls + rand, dtype=np.int64)


def main():
    P, F = W.shock_tube(512, 1024, 2000)
    g = O.Grid(P.nr, P.nth, P.r1, P.r2, P.tau, P.dt, P.bc_kind, P.bc_par)
    f0 = O.init_feq(g, **F)
    nodes = sample_nodes(P.nr, P.nth, 376, 2024)
    a = f0.copy()
    b = f0.copy()
    rng = np.random.default_rng(7)
    bad = 0
    for s in range(P.steps):
        a, ba = O.step(g, a, 1)
        b, _ = O.step(g, b, 1)
        b *= 1.0 + NOISE_ULPS * 2.0 ** -52 * rng.uniform(-1.0, 1.0, b.shape)
        bad += ba
        if (s + 1) % 200 == 0:
            print(f"step {s + 1}", flush=True)
    rho, ur, ut, T = O.fields(g, a)
    prof = np.stack([np.stack([x.mean(1), x.min(1), x.max(1)]) for x in (rho, ur, ut, T)])
    np.savez_compressed(
        OUT, steps=P.steps, dt=P.dt, tau=P.tau, nodes=nodes,
        f_nodes=a[:, nodes[:, 0], nodes[:, 1]].T, f_nodes_noisy=b[:, nodes[:, 0], nodes[:, 1]].T,
        noise_floor=np.linalg.norm(b - a) / np.linalg.norm(a),
        profiles=prof, diagnostics=O.diagnostics(g, a), bad_ghosts=bad)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
