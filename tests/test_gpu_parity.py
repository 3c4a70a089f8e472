"""GPU path (libstbem.so through the C ABI) against the CPU oracle.

Entries: |A_gpu - A_ref| <= tol * max(|A_ref|, 1e-8 * max over the block of
|A_ref|), tol = 1e-12 for every operator.  Solutions: relative l2 error <= 1e-10
against the oracle's direct block forward substitution on the oracle's own
matrices.
"""
import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle, packed_apply, packed_index

pytestmark = pytest.mark.gpu

TOL = {"V": 1e-12, "K": 1e-12, "D": 1e-12, "dV": 1e-12, "dK": 1e-12}


def _ctx(wl, mask):
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    c = P.Context.from_workload(wl)
    c.assemble(mask)
    return c, L


def block_err(gpu, ref):
    """floor-rule relative error per entry of packed [nb, ng, ng] arrays"""
    mx = np.abs(ref).reshape(ref.shape[0], -1).max(axis=1)[:, None, None]
    return np.abs(gpu - ref) / np.maximum(np.abs(ref), 1e-8 * mx + 1e-300)


@pytest.fixture(scope="module")
def small():
    # 20 segments: two 16-wide tiles per block side, the second one ragged
    wl = W.make("custom", n_side=5, n_t=4, n_omega=3, alpha=1.3, k=(0.4, -0.3))
    o = Oracle.from_workload(wl)
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    c = P.Context.from_workload(wl)
    c.assemble(L.V | L.K | L.D | L.M0 | L.DV | L.DK | L.DM0)
    return wl, o, c, L


@pytest.mark.parametrize("op", ["V", "K", "D", "dV", "dK"])
def test_assembly_small_all_entries(small, op):
    wl, o, c, L = small
    code = {"V": L.V, "K": L.K, "D": L.D, "dV": L.DV, "dK": L.DK}[op]
    gpu = c.packed(code).cpu().numpy()
    ref = o.packed(op)
    e = block_err(gpu, ref)
    print(op, "max floor-rule error", e.max())
    assert e.max() <= TOL[op]


def test_symmetric_blocks_stored_exactly_symmetric(small):
    """V_h, dV_h/dalpha and D_h blocks are symmetric in space; the kernels
    compute the tiles on and above the block diagonal and store the mirror,
    so every stored block equals its transpose bit for bit (K_h is not
    symmetric and is not mirrored)."""
    wl, o, c, L = small
    for code in (L.V, L.DV, L.D):
        P = c.packed(code).cpu().numpy()
        assert np.array_equal(P, np.transpose(P, (0, 2, 1)))
    Kp = c.packed(L.K).cpu().numpy()
    assert not np.array_equal(Kp, np.transpose(Kp, (0, 2, 1)))


def test_launch_timing_records(small):
    """The launch timing of the library reports every assembly kernel of a
    V_h + D_h + K_h assembly with its work units (matrix entries of the
    blocks it processed) and a positive event time; switching it off drops
    the records.  Assembled together, V_h's blocks come from D_h's tile
    launches (named "k_assemble_dfar<q, true, true>" and
    "k_assemble_dnear<true>"), which count their D_h entries; the V_h entries
    they write are the same number, and so are the K_h entries of the far
    tiles (K_h's touching blocks and the blocks outside D_h's far lists go
    through K_h's own kernels)."""
    wl, o, c, L = small
    c.set_timing(True)
    c.assemble(L.V | L.K | L.D)
    rec = c.kernel_times()
    c.set_timing(False)
    assert c.kernel_times() == {}
    entries = c.packed_entries
    by_op = {"V": ("k_assemble<0>", "k_assemble_vkfar<0,"), "K": ("k_assemble_knear<1>", "k_assemble<1>", "k_assemble_vkfar<1,"),
             "D": ("k_assemble_dnear", "k_assemble<2>", "k_assemble_dfar<")}
    fused = sum(u for name, (n, ms, u, fl) in rec.items()
                if name.startswith(("k_assemble_dfar<", "k_assemble_dnear<")) and name.endswith("true>"))
    assert fused > 0
    fused_k = sum(u for name, (n, ms, u, fl) in rec.items()
                  if name.startswith("k_assemble_dfar<") and name.endswith("true, true>"))
    assert fused_k > 0
    extra = {"V": fused, "K": fused_k, "D": 0}
    for op, prefixes in by_op.items():
        units = sum(u for name, (n, ms, u, fl) in rec.items() if name.startswith(prefixes))
        assert units + extra[op] == entries, (op, units, entries)
    for name, (n, ms, u, fl) in rec.items():
        assert n >= 1 and ms > 0.0 and u > 0, name


@pytest.mark.parametrize("deriv", [False, True])
def test_m0_small_all_entries(small, deriv):
    wl, o, c, L = small
    gpu = c.matrix(L.DM0 if deriv else L.M0).cpu().numpy().reshape(c.n, c.nv)
    ref = o.m0(deriv)
    mx = np.abs(ref).max(axis=1, keepdims=True)
    e = np.abs(gpu - ref) / np.maximum(np.abs(ref), 1e-8 * mx)
    print("M0 max error", e.max())
    assert e.max() <= 1e-12


def test_sampled_entries_kernel_matches_storage(small):
    wl, o, c, L = small
    rng = np.random.default_rng(3)
    idx = np.stack([rng.integers(0, c.nt, 64), rng.integers(0, c.nt, 64), rng.integers(0, c.ng, 64), rng.integers(0, c.ng, 64)], 1)
    idx[:, 1] = np.minimum(idx[:, 0], idx[:, 1])
    for code in (L.V, L.K, L.D):
        a = c.entries(code, idx).cpu().numpy()
        P = c.packed(code).cpu().numpy()
        b = np.array([P[packed_index(k, m), i, j] for k, m, i, j in idx])
        # separated time blocks are stored by the far-field kernels (shared
        # piece moments, unrolled node loops): same integrals, other
        # summation order than the per-entry kernel
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15 * np.abs(b).max())


def test_gemv_matches_numpy_and_is_deterministic(small):
    wl, o, c, L = small
    rng = np.random.default_rng(5)
    x = rng.standard_normal(c.n)
    for code in (L.V, L.K, L.D):
        P = c.packed(code).cpu().numpy()
        for trans in (False, True):
            y1 = c.apply(code, x, trans=trans).cpu().numpy()
            y2 = c.apply(code, x, trans=trans).cpu().numpy()
            ref = packed_apply(P, x, c.nt, c.ng, trans=trans)
            assert np.array_equal(y1, y2)
            assert np.abs(y1 - ref).max() <= 1e-14 * np.abs(P).max() * np.abs(x).sum() ** 0.5 * c.n ** 0.5
    M0 = c.matrix(L.M0).cpu().numpy().reshape(c.n, c.nv)
    u = rng.standard_normal(c.nv)
    np.testing.assert_allclose(c.apply(L.M0, u).cpu().numpy(), M0 @ u, rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(c.apply(L.M0, x, trans=True).cpu().numpy(), M0.T @ x, rtol=1e-13, atol=1e-16)


def test_rhs_and_solves_small(small):
    wl, o, c, L = small
    V, K, D, M0 = o.packed("V"), o.packed("K"), o.packed("D"), o.m0()
    f_ref = o.rhs(K, M0, wl.g, wl.u0)
    f = c.rhs(wl.g, wl.u0).cpu().numpy()
    assert np.linalg.norm(f - f_ref) / np.linalg.norm(f_ref) < 1e-12
    w_ref = o.solve_direct(V, f_ref)
    for mode in (L.FP64, L.FP32_IR):
        w, info = c.solve(f_ref, tol=1e-13, max_it=200, mode=mode, ir_tol=1e-13)
        err = np.linalg.norm(w.cpu().numpy() - w_ref) / np.linalg.norm(w_ref)
        print("mode", mode, "iters", info.iters, "outer", info.outer, "err", err, "true relres", info.true_relres)
        assert err < 1e-10
        assert info.status == 0
    # adjoint solve: V^T lam = f
    lam, info = c.solve(f_ref, tol=1e-13, max_it=200, trans=True)
    lam_ref = o.solve_direct(V, f_ref) if False else None
    import scipy.linalg as sla
    A = o.dense(V)
    lam_ref = sla.solve(A.T, f_ref)
    assert np.linalg.norm(lam.cpu().numpy() - lam_ref) / np.linalg.norm(lam_ref) < 1e-10


@pytest.fixture(scope="module")
def tiny():
    wl = W.make("tiny")
    o = Oracle.from_workload(wl)
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    c = P.Context.from_workload(wl)
    c.assemble(L.V | L.K | L.D | L.M0)
    return wl, o, c, L


@pytest.mark.parametrize("op", ["V", "K", "D"])
def test_tiny_all_entries(tiny, op):
    wl, o, c, L = tiny
    code = {"V": L.V, "K": L.K, "D": L.D}[op]
    e = block_err(c.packed(code).cpu().numpy(), o.packed(op))
    print(op, "tiny max floor-rule error", e.max())
    assert e.max() <= TOL[op]


def test_tiny_solution(tiny):
    wl, o, c, L = tiny
    V, K, M0 = o.packed("V"), o.packed("K"), o.m0()
    f_ref = o.rhs(K, M0, wl.g, wl.u0)
    w_ref = o.solve_direct(V, f_ref)
    f = c.rhs(wl.g, wl.u0)
    w, info = c.solve(f, tol=1e-13, max_it=200)
    err = np.linalg.norm(w.cpu().numpy() - w_ref) / np.linalg.norm(w_ref)
    print("tiny solve iters", info.iters, "err vs oracle", err)
    assert err < 1e-10


def test_assembled_alone_or_together(small):
    """V_h, K_h and D_h assembled in one call share D_h's tiles (V_h's and
    K_h's separated blocks come from the same piece pairs, V_h's touching
    blocks too); assembled alone each uses its own kernels.  Both ways must
    meet the oracle bar, and agree with each other to the quadrature level;
    D_h's own arithmetic is the same either way."""
    wl, o, c, L = small
    import paper_1811_05224_amd as P
    alone = {}
    for code in (L.V, L.K, L.D):
        ca = P.Context.from_workload(wl)
        ca.assemble(code)
        alone[code] = ca.packed(code).cpu().numpy()
        ca.close()
    for code, op in ((L.V, "V"), (L.K, "K"), (L.D, "D")):
        fused = c.packed(code).cpu().numpy()
        ref = o.packed(op)
        ea, ef = block_err(alone[code], ref).max(), block_err(fused, ref).max()
        diff = np.abs(alone[code] - fused).max() / np.abs(fused).max()
        print(op, "alone vs oracle", ea, "together vs oracle", ef, "alone vs together", diff)
        assert ea <= TOL[op] and ef <= TOL[op]
        assert diff <= 1e-13
    assert np.array_equal(alone[L.V], np.transpose(alone[L.V], (0, 2, 1)))


def test_preconditioner_matches_oracle(small):
    """stbem_precondition is C_V^{-1} r = Mt^{-1} D_h Mt^{-1} r (Thm 1 with the
    lumped dual mass of Sec. 4): against the oracle's D_h and its lumped
    mass (row sums of the dual-primal mass matrix), both directions."""
    wl, o, c, L = small
    D = o.packed("D")
    mt = o.lumped_dual_mass()
    rng = np.random.default_rng(9)
    r = rng.standard_normal(c.n)
    for trans in (False, True):
        z = c.precondition(r, trans=trans).cpu().numpy()
        ref = packed_apply(D, r / mt, c.nt, c.ng, trans=trans) / mt
        err = np.abs(z - ref).max() / np.abs(ref).max()
        print("trans", trans, "preconditioner error", err)
        assert err <= 1e-12


@pytest.mark.parametrize("precondition", [True, False])
def test_iteration_counts_match_oracle_gmres(small, precondition):
    """The GPU's GMRES and the oracle's (same left preconditioning, x0 = 0,
    no restart, same stopping rule on the preconditioned residual) take the
    same number of iterations on the oracle's right-hand side."""
    wl, o, c, L = small
    V, D, K, M0 = o.packed("V"), o.packed("D"), o.packed("K"), o.m0()
    f = o.rhs(K, M0, wl.g, wl.u0)
    for tol in (1e-6, 1e-10):
        _, it_o, hist = o.solve_gmres(V, D, f, tol=tol, precondition=precondition)
        _, info = c.solve(f, tol=tol, max_it=200, precondition=precondition)
        print("precondition", precondition, "tol", tol, "oracle", it_o, "gpu", info.iters)
        # both stop at the first iterate below tol; only a residual within
        # rounding of tol could split them
        near = any(abs(h / tol - 1) < 1e-6 for h in hist)
        assert info.iters == it_o or (near and abs(info.iters - it_o) <= 1)
