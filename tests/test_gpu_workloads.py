"""Parity on the large workloads at their full sizes, in the configuration
bench.py times (the precision workload is its default).

precision: unit square, 512 segments x 256 uniform steps (N = 131072);
  K_h and M_h^0 (69 + 17.4 GB) are released once the right-hand side is
  formed; V_h and D_h in FP64 (69 GB each), then released and assembled
  again into FP32 storage (V_h as the pair hi + lo, D_h as FP32: 103.5 GB).
lshape:    [0,1]^2 minus [0.5,1]^2, 384 segments, 200 geometric steps
  (ratio 1.02, finest at t = 0), alpha = 0.1 (no block-Toeplitz structure).

Entries are sampled and compared one by one with the oracle (floor rule as
in the small tests); solutions are checked through the residual in rows
that the oracle assembles, for the FP64 and the FP32-refined solve, and both
solutions at the benchmark's tolerances must be within 1e-10 (relative l2)
of an FP64 solve to 1e-15.
"""
import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle
from floor_rule import block_floor

pytestmark = pytest.mark.gpu


def _sample(ng, nt, rng, nblocks):
    blocks = [(int(k), int(k)) for k in rng.integers(0, nt, 3)] + \
             [(int(k), int(max(k - 1, 0))) for k in rng.integers(1, nt, 3)] + \
             [(int(k), int(rng.integers(0, k + 1))) for k in rng.integers(0, nt, nblocks)] + [(nt - 1, 0)]
    idx = []
    for (k, m) in blocks:
        i = int(rng.integers(0, ng))
        cols = {i, (i + 1) % ng, (i - 1) % ng, (i + 3) % ng, (i + ng // 3) % ng, int(rng.integers(0, ng))}
        idx += [(k, m, i, j) for j in sorted(cols)]
    return np.array(idx, dtype=np.int32)


def _check_entries(c, o, op, code, idx, tol):
    import torch
    ref = o.entries(op, idx)
    P = c.packed(code)
    b = idx[:, 0].astype(np.int64) * (idx[:, 0] + 1) // 2 + idx[:, 1]
    t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.int64), device=P.device)
    got = P[t(b), t(idx[:, 2]), t(idx[:, 3])].cpu().numpy()
    floor = block_floor(o, op, idx, ref, c.ng)
    e = np.abs(got - ref) / np.maximum(np.abs(ref), floor + 1e-300)
    print(op, "samples", len(idx), "max err", e.max())
    for w in np.argsort(e)[::-1][:6]:
        if e[w] > tol:
            print("   ", tuple(int(x) for x in idx[w]), "gpu", got[w], "oracle", ref[w])
    assert e.max() <= tol


def _row_data(o, c, wl, rows):
    data = []
    for (k, i) in rows:
        idx = np.array([(k, m, i, j) for m in range(k + 1) for j in range(c.ng)], dtype=np.int32)
        cols = idx[:, 1] * c.ng + idx[:, 3]
        mrow = np.zeros(c.n)
        mrow[k * c.ng + i] += 0.5 * o.h[k] * o.L[i]
        mrow[k * c.ng + (i + 1) % c.ng] += 0.5 * o.h[k] * o.L[i]
        data.append((cols, o.entries("V", idx), o.entries("K", idx), mrow, o.m0_rows([(k, i)])[0]))
    return data


def _check_rows(wl, wn, rows, data, tol=1e-10):
    for (k, i), (cols, vrow, krow, mrow, m0row) in zip(rows, data):
        lhs = vrow @ wn[cols]
        rhs = 0.5 * (mrow @ wl.g) + krow @ wl.g[cols] - m0row @ wl.u0
        scale = np.abs(vrow) @ np.abs(wn[cols]) + np.abs(krow) @ np.abs(wl.g[cols]) + np.abs(m0row) @ np.abs(wl.u0)
        print("row", (k, i), "residual/scale", abs(lhs - rhs) / scale)
        assert abs(lhs - rhs) <= tol * scale


@pytest.mark.parametrize("name", ["lshape", "precision"])
def test_large_workload(name):
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    wl = W.make(name, seed=0)
    o = Oracle.from_workload(wl)
    c = P.Context.from_workload(wl)
    rng = np.random.default_rng(11)
    rows = [(1, 5), (int(c.nt * 0.4), c.ng // 2), (c.nt - 1, c.ng // 4 + 3)]
    data = _row_data(o, c, wl, rows)
    c.assemble(L.K | L.M0)
    f = c.rhs(wl.g, wl.u0)
    _check_entries(c, o, "K", L.K, _sample(c.ng, c.nt, rng, 6), 1e-12)
    c.release(L.K | L.M0)
    c.assemble(L.V | L.D)
    _check_entries(c, o, "V", L.V, _sample(c.ng, c.nt, rng, 8), 1e-12)
    _check_entries(c, o, "D", L.D, _sample(c.ng, c.nt, rng, 4), 1e-12)
    # the benchmark's tolerances (bench.py defaults) and a tight reference
    w64, i64 = c.solve(f, tol=3e-11, max_it=400)
    assert i64.status == 0
    wref, iref = c.solve(f, tol=1e-15, max_it=800)
    c.release(L.V | L.D)
    c.assemble(L.V | L.D, precision=L.FP32_IR)
    _check_f32_entries(c, o, L, _sample(c.ng, c.nt, rng, 6))
    w32, i32 = c.solve(f, tol=1e-12, max_it=400, mode=L.FP32_IR, inner_tol=1e-6, max_outer=12, ir_tol=1e-12)
    assert i32.status == 0
    w64n, w32n, wrn = w64.cpu().numpy(), w32.cpu().numpy(), wref.cpu().numpy()
    e64 = np.linalg.norm(w64n - wrn) / np.linalg.norm(wrn)
    e32 = np.linalg.norm(w32n - wrn) / np.linalg.norm(wrn)
    print(name, "GMRES iters", i64.iters, "(reference", iref.iters, ") IR inner", i32.iters, "outer", i32.outer,
          "err fp64", e64, "err fp32-refined", e32)
    assert e64 <= 1e-10 and e32 <= 1e-10
    _check_rows(wl, w64n, rows, data)
    _check_rows(wl, w32n, rows, data)
    c.close()


def _check_f32_entries(c, o, L, idx):
    """FP32 storage: V_h's pair hi + lo at the FP64 bar, D_h at FP32 rounding."""
    import torch
    b = idx[:, 0].astype(np.int64) * (idx[:, 0] + 1) // 2 + idx[:, 1]
    t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.int64), device=c.device)
    # D_h: FP32 arithmetic on separated time blocks, so its bar is taken
    # against a floor of 1e-3 of the sampled block maximum as well
    for op, code, tol in (("V", L.V, 1e-12), ("D", L.D, 2e-6)):
        hi, lo = c.packed_f32(code)
        got = hi[t(b), t(idx[:, 2]), t(idx[:, 3])].double()
        if lo is not None:
            got = got + lo[t(b), t(idx[:, 2]), t(idx[:, 3])].double()
        got = got.cpu().numpy()
        ref = o.entries(op, idx)
        floor = block_floor(o, op, idx, ref, c.ng)
        if op == "D":
            floor = 1e5 * floor           # 1e-3 of the sampled block maximum
        e = np.abs(got - ref) / np.maximum(np.abs(ref), floor + 1e-300)
        print(op, "fp32 storage, samples", len(idx), "max err", e.max())
        assert e.max() <= tol
