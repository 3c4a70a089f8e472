"""Writes the oracle's GMRES iteration counts for the experiment of Sec. 4
(Table 1) at L = 2 and 3: the paper's sine solution, alpha = 10, uniform
meshes, GMRES to 1e-8 without and with the D_h preconditioner
(M~^-1 D_h M~^-1, lumped dual mass), all from oracle/.

Run from the repository root:  python tests/golden/make_table1_oracle.py
(about 10 minutes on 8 cores).  Output: tests/golden/table1_oracle_counts.txt
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.oracle import Oracle, packed_apply  # noqa: E402


def counts(L):
    wl = W.paper_level(L)
    o = Oracle.from_workload(wl)
    V, K, D = o.packed("V"), o.packed("K"), o.packed("D")
    f = o.rhs(K, o.m0(), wl.g, wl.u0)
    _, it_plain, _ = o.solve_gmres(V, D, f, tol=1e-8, precondition=False)
    _, it_prec, _ = o.solve_gmres(V, D, f, tol=1e-8, precondition=True)
    return o.n, it_plain, it_prec


if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "table1_oracle_counts.txt")
    lines = ["# Oracle GMRES iteration counts for the experiment of Sec. 4 (Table 1),",
             "# written by make_table1_oracle.py (oracle only): L  N  plain  preconditioned"]
    for L in (2, 3):
        t0 = time.time()
        n, a, b = counts(L)
        print(f"L={L} N={n}: {a} plain, {b} preconditioned ({time.time() - t0:.0f} s)", flush=True)
        lines.append(f"{L} {n} {a} {b}")
    open(out, "w").write("\n".join(lines) + "\n")
