"""The oracle's singular entries against an independent brute force.

Touching time elements (d = k - m in {0, 1}) with coincident or
vertex-sharing pieces are where the Galerkin entries of eq.(4) (and of D_h
in the integration-by-parts form of Sec. 2) are singular, and where the
oracle uses its special quadrature (difference variable, Duffy split,
polar coordinates for M_h^0's first time step).  ``tests/bruteforce.py``
integrates the raw fundamental solution there with different rules (exact
lag reduction of the time integral, numerical in ln s; hp-graded Gauss in
space); it shares nothing with ``oracle/``.
"""
import concurrent.futures as cf
import multiprocessing as mpr

import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle

import bruteforce as B

ALPHA = 1.3
# graded steps: the first elements are short, so d = 0 and 1 are met at
# several step ratios
T_NODES = W.graded_times(5, 1.6)
BND = W.square_polygon(4)          # 16 segments, corners at vertices 0, 4, 8, 12

# (k, m): d = 0 on the shortest and on a longer element, d = 1 at ratio
# 1.6, and one separated pair (d = 2) as a control
BLOCKS = [(0, 0), (3, 3), (1, 0), (4, 3), (2, 0)]
PAIRS = {
    # V: coincident, collinear neighbours, neighbours at the corner x_4
    "V": [(1, 1), (1, 2), (3, 4)],
    # K (column = hat of polygon vertex n on segments n-1, n): the corner hat
    # seen from both adjacent segments, and the hat next to the corner
    "K": [(3, 4), (4, 4), (3, 5), (2, 4)],
    # D (dual hats at segment midpoints): same function, neighbours on one
    # side and across the corner, next-but-one across the corner
    "D": [(1, 1), (1, 2), (3, 4), (4, 4), (3, 5)],
}


def _pool():
    return cf.ProcessPoolExecutor(max_workers=8, mp_context=mpr.get_context("spawn"))


@pytest.mark.parametrize("op", ["V", "K", "D"])
def test_singular_entries_vs_raw_kernel(op):
    """V_h, K_h, D_h entries on touching time elements (and one separated
    control block) agree with the brute force to 1e-11 relative, with a
    floor of 1e-13 of the block's largest entry among those checked
    (entries of D between neighbouring dual hats nearly cancel)."""
    idx = [(k, mm, i, j) for (k, mm) in BLOCKS for (i, j) in PAIRS[op]]
    got = Oracle(ALPHA, T_NODES, BND).entries(op, idx)
    with _pool() as ex:
        ref = np.array(list(ex.map(B.entry_packed, [(ALPHA, T_NODES, BND, op, *q) for q in idx])))
    for b in range(len(BLOCKS)):
        sl = slice(b * len(PAIRS[op]), (b + 1) * len(PAIRS[op]))
        scale = np.abs(ref[sl]).max()
        err = np.abs(got[sl] - ref[sl])
        bound = 1e-11 * np.abs(ref[sl]) + 1e-13 * scale
        assert np.all(err <= bound), (op, BLOCKS[b], err / np.maximum(np.abs(ref[sl]), 1e-300))


def test_m0_singular_rows_vs_bruteforce():
    """M_h^0 entries of the first two time steps (k = 0: log-singular time
    kernel on triangles touching the segment) against the brute force:
    the corner hat, hats whose support touches the segment only at its end
    point, and a hat with an edge on the segment; 1e-12 relative."""
    wl = W.make("tiny")
    o = Oracle.from_workload(wl)
    m = B.Mesh(wl.alpha, wl.t_nodes, wl.bnd_xy)
    cases = [(0, 0, 0), (0, 1, 1), (0, 1, 2), (0, 1, 10), (1, 1, 1), (1, 0, 9)]
    keys = sorted({(k, i) for (k, i, _) in cases})
    rows = dict(zip(keys, o.m0_rows(keys)))
    args = []
    for (k, i, j) in cases:
        seg = m.seg(i)
        args.append((wl.alpha, wl.t_nodes, k, seg.a, seg.e, seg.L, wl.tri, wl.vtx_xy, j))
    with _pool() as ex:
        ref = list(ex.map(B.m0_entry_packed, args))
    for (k, i, j), r in zip(cases, ref):
        got = rows[(k, i)][j]
        assert got == pytest.approx(r, rel=1e-12), (k, i, j, got, r)
