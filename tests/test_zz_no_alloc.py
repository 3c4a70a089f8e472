"""stbem_apply_noalloc (the entry point for callers that cannot allocate)
against stbem_apply, through the C ABI.

Two calls in a row on one GPU, the second with a smaller problem: first the
Table 2 mesh (512 segments x 128 steps, whose 8256 x 512 partials exceed the
32 MiB buffer, so the block rows go in two ranges), then the 16 x 16 mesh
(one range).  trans = 0 must equal stbem_apply bitwise; trans = 1 too with
one range, and to rounding of the additions with two.
"""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

SCRATCH_DOUBLES = (32 << 20) // 8


def _noalloc(c, op, x, trans):
    y = torch.full((c.n,), float("nan"), dtype=torch.float64, device=c.device)
    rc = c.lib.stbem_apply_noalloc(c._h, int(op), int(trans), ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(y.data_ptr()), c._stream())
    assert rc == 0, c.lib.stbem_last_error(c._h)
    return y


def _check(c, op, x, ranges_one):
    from paper_1811_05224_amd import _lib as L  # noqa: F401
    for trans in (0, 1):
        ref = c.apply(op, x, trans=bool(trans)).cpu().numpy()
        got = _noalloc(c, op, x, trans).cpu().numpy()
        assert np.all(np.isfinite(got))
        if trans == 0 or ranges_one:
            assert np.array_equal(got, ref), (op, trans, np.abs(got - ref).max())
        else:
            err = np.abs(got - ref).max() / np.abs(ref).max()
            assert err <= 1e-14, (op, trans, err)


def test_noalloc_apply_matches_apply_two_calls():
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    torch.manual_seed(0)
    # call 1: two ranges of block rows
    wl = W.paper_level(7)
    c = P.Context.from_workload(wl)
    assert c.nt * (c.nt + 1) // 2 * c.ng > SCRATCH_DOUBLES >= c.nt * c.ng
    c.assemble(L.V)
    x = torch.randn(c.n, dtype=torch.float64, device=c.device)
    print("noalloc: paper mesh 512 x 128, V_h", flush=True)
    _check(c, L.V, x, ranges_one=False)
    c.close()
    del c
    torch.cuda.empty_cache()
    # call 2: a smaller problem on the same buffer, FP64 and FP32 storage
    wl = W.make("tiny")
    c = P.Context.from_workload(wl)
    c.assemble(L.V | L.K | L.D)
    x = torch.randn(c.n, dtype=torch.float64, device=c.device)
    for op in (L.V, L.K, L.D):
        print("noalloc: tiny, op", op, flush=True)
        _check(c, op, x, ranges_one=True)
    c.assemble(L.V | L.D, precision=L.FP32_IR)
    for op in (L.V, L.D):
        print("noalloc: tiny FP32 storage, op", op, flush=True)
        _check(c, op, x, ranges_one=True)
    # refused: dense operator, unassembled operator
    y = torch.empty(c.n, dtype=torch.float64, device=c.device)
    assert c.lib.stbem_apply_noalloc(c._h, int(L.M0), 0, ctypes.c_void_p(x.data_ptr()),
                                     ctypes.c_void_p(y.data_ptr()), c._stream()) == -1
    assert c.lib.stbem_apply_noalloc(c._h, int(L.DV), 0, ctypes.c_void_p(x.data_ptr()),
                                     ctypes.c_void_p(y.data_ptr()), c._stream()) == -6
    c.close()
