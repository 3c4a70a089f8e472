"""Writes reference solutions of eq.(4) computed by the oracle alone.

For each case: the Dirichlet data g of the manufactured solution
exp(k.x + |k|^2 t/alpha) (workloads.py), u0 = 0, the right-hand side
f = (1/2 M_h + K_h) g, and w solving V_h w = f by block forward
substitution (Cholesky of the symmetric positive definite diagonal block),
all from oracle/.  Uniform steps use the oracle's block-Toeplitz blocks
(d, 0); the graded case assembles the whole lower block triangle.

Run from the repository root:  python tests/golden/make_reference_solutions.py
(about 45 minutes on 8 cores).  Output: tests/golden/solution_<case>.npz with
arrays f, w and the case parameters (plain float64; load with numpy.load,
allow_pickle=False).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.oracle import (Oracle, packed_apply, block_forward_solve,  # noqa: E402
                           toeplitz_apply, toeplitz_forward_solve)

CASES = {
    # the differentiation workload's mesh: 128 segments x 128 uniform steps
    "square128_uniform": dict(bnd=lambda: W.square_polygon(32), t=lambda: W.uniform_times(128), alpha=1.0,
                              k=(1.0, 0.0)),
    # L-shape, 48 segments x 32 geometrically graded steps (ratio 1.1), alpha = 0.1
    "lshape48_graded": dict(bnd=lambda: W.lshape_polygon(48), t=lambda: W.graded_times(32, 1.1), alpha=0.1,
                            k=(0.8, -1.1)),
}


def make(name):
    cfg = CASES[name]
    bnd, t, alpha = cfg["bnd"](), cfg["t"](), cfg["alpha"]
    vx, _ = W.square_grid(2)
    g, _, _ = W.manufactured(bnd, t, vx, alpha, np.asarray(cfg["k"], dtype=np.float64))
    o = Oracle(alpha, t, bnd)
    nt, ng = o.nt, o.ng
    t0 = time.time()
    h = np.diff(t)
    if np.abs(h - h[0]).max() <= 1e-12 * h[0]:
        Vt, Kt = o.toeplitz_blocks("V"), o.toeplitz_blocks("K")
        f = 0.5 * o.mass_apply(g) + toeplitz_apply(Kt, g, nt, ng)
        w = toeplitz_forward_solve(Vt, f, nt, ng)
        res = np.linalg.norm(toeplitz_apply(Vt, w, nt, ng) - f) / np.linalg.norm(f)
    else:
        V, K = o.packed("V"), o.packed("K")
        f = 0.5 * o.mass_apply(g) + packed_apply(K, g, nt, ng)
        w = block_forward_solve(V, f, nt, ng)
        res = np.linalg.norm(packed_apply(V, w, nt, ng) - f) / np.linalg.norm(f)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"solution_{name}.npz")
    np.savez(out, f=f, w=w, g=g, alpha=alpha, t_nodes=t, bnd_xy=bnd)
    print(f"{name}: N = {o.n}, residual {res:.1e}, {time.time() - t0:.0f} s -> {out}", flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES)):
        make(name)
