"""Parity at the benchmark's full size (medium: 256 segments x 128 steps,
N = 32768, Omega 64^2), in the configuration bench.py times.

Entries: stratified samples (touching/separated time elements, coincident,
adjacent, near and far spatial pairs) compared with the oracle one by one;
the floor of the relative error is 1e-8 of the block's scale (the oracle's
largest sampled value, for K_h its largest value in the sampled row).
Solution: the oracle evaluates single rows of V_h, K_h, M_h and M_h^0 and
checks the residual of the GPU solution row by row.
"""
import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle
from floor_rule import block_floor

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def medium():
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    wl = W.make("medium")
    c = P.Context.from_workload(wl)
    c.assemble(L.V | L.K | L.D | L.M0)
    return wl, Oracle.from_workload(wl), c, L


def _sample(ng, nt, rng, nblocks=24):
    ks = list(rng.integers(0, nt, nblocks))
    blocks = [(k, k) for k in ks[:6]] + [(k, max(k - 1, 0)) for k in ks[6:12]] + \
             [(k, int(rng.integers(0, k + 1))) for k in ks[12:]] + [(nt - 1, 0)]
    idx = []
    for (k, m) in blocks:
        i = int(rng.integers(0, ng))
        cols = {i, (i + 1) % ng, (i - 1) % ng, (i + 2) % ng, (i + 5) % ng, (i + ng // 2) % ng,
                int(rng.integers(0, ng)), int(rng.integers(0, ng))}
        idx += [(k, m, i, j) for j in sorted(cols)]
    return np.array(idx, dtype=np.int32)


@pytest.mark.parametrize("op,tol", [("V", 1e-12), ("K", 1e-12), ("D", 1e-12)])
def test_medium_sampled_entries(medium, op, tol):
    wl, o, c, L = medium
    rng = np.random.default_rng({"V": 1, "K": 2, "D": 3}[op])
    idx = _sample(c.ng, c.nt, rng)
    ref = o.entries(op, idx)
    P = c.packed({"V": L.V, "K": L.K, "D": L.D}[op])
    import torch
    b = idx[:, 0].astype(np.int64) * (idx[:, 0] + 1) // 2 + idx[:, 1]
    t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.int64), device=P.device)
    got = P[t(b), t(idx[:, 2]), t(idx[:, 3])].cpu().numpy()
    floor = block_floor(o, op, idx, ref, c.ng)
    e = np.abs(got - ref) / np.maximum(np.abs(ref), floor + 1e-300)
    print(op, "samples", len(idx), "max err", e.max())
    assert e.max() <= tol


def test_medium_m0_rows(medium):
    wl, o, c, L = medium
    rows = [(0, 0), (0, 37), (0, 130), (1, 64), (5, 200), (60, 255), (127, 100)]
    ref = o.m0_rows(rows)
    M0 = c.matrix(L.M0).view(c.n, c.nv)
    got = np.stack([M0[k * c.ng + i].cpu().numpy() for k, i in rows])
    mx = np.abs(ref).max(axis=1, keepdims=True)
    e = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-8 * mx)
    print("M0 rows max err", e.max())
    assert e.max() <= 1e-12


def test_medium_solution_rows(medium):
    """Residual of the GPU solution in rows assembled by the oracle:
    |(V w - (1/2 M + K) g + M0 u0)_l| <= 1e-10 * sum_j |V_lj w_j| (+ the
    same for the right-hand side terms)."""
    wl, o, c, L = medium
    f = c.rhs(wl.g, wl.u0)
    rows = [(0, 3), (17, 128), (127, 255)]
    data = []
    for (k, i) in rows:
        idx = np.array([(k, m, i, j) for m in range(k + 1) for j in range(c.ng)], dtype=np.int32)
        cols = idx[:, 1] * c.ng + idx[:, 3]
        mrow = np.zeros(c.n)
        mrow[k * c.ng + i] += 0.5 * o.h[k] * o.L[i]
        mrow[k * c.ng + (i + 1) % c.ng] += 0.5 * o.h[k] * o.L[i]
        data.append((cols, o.entries("V", idx), o.entries("K", idx), mrow, o.m0_rows([(k, i)])[0]))
    for mode in (L.FP64, L.FP32_IR):
        w, info = c.solve(f, tol=1e-12, max_it=300, mode=mode, ir_tol=1e-12)
        assert info.status == 0
        wn = w.cpu().numpy()
        for (k, i), (cols, vrow, krow, mrow, m0row) in zip(rows, data):
            lhs = vrow @ wn[cols]
            rhs = 0.5 * (mrow @ wl.g) + krow @ wl.g[cols] - m0row @ wl.u0
            scale = np.abs(vrow) @ np.abs(wn[cols]) + np.abs(krow) @ np.abs(wl.g[cols]) + np.abs(m0row) @ np.abs(wl.u0)
            print("mode", mode, "row", (k, i), "residual/scale", abs(lhs - rhs) / scale)
            assert abs(lhs - rhs) <= 1e-10 * scale


def test_medium_bench_tolerances_reach_1e10(medium):
    """The solve tolerances bench.py times with (FP64 GMRES to a 3e-11
    preconditioned residual; FP32-stored refinement to a 1e-12 FP64 residual
    with 1e-6 inner solves) give solutions within 1e-10 (relative l2) of an
    FP64 solve to 1e-15, whose residual against oracle rows is checked by
    test_medium_solution_rows."""
    wl, o, c, L = medium
    f = c.rhs(wl.g, wl.u0)
    wref, iref = c.solve(f, tol=1e-15, max_it=800)
    nr = float(np.linalg.norm(wref.cpu().numpy()))
    w64, i64 = c.solve(f, tol=3e-11, max_it=400)
    w32, i32 = c.solve(f, tol=1e-12, max_it=400, mode=L.FP32_IR, inner_tol=1e-6, max_outer=12, ir_tol=1e-12)
    assert i64.status == 0 and i32.status == 0
    e64 = float(np.linalg.norm((w64 - wref).cpu().numpy())) / nr
    e32 = float(np.linalg.norm((w32 - wref).cpu().numpy())) / nr
    print("FP64", i64.iters, "iterations, error", e64, "; FP32-refined", i32.outer, "outer", i32.iters, "inner, error", e32)
    assert e64 <= 1e-10 and e32 <= 1e-10
