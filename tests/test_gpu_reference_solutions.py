"""GPU solutions against stored oracle solutions on meshes above the tiny one.

``tests/golden/make_reference_solutions.py`` (oracle only) wrote, for the
differentiation workload's mesh (128 segments x 128 uniform steps,
N = 16384) and for an L-shape with 48 segments x 32 graded steps
(alpha = 0.1, N = 1536), the right-hand side f = (1/2 M_h + K_h) g of eq.(4)
for manufactured Dirichlet data g, u0 = 0, and the solution w of V_h w = f
by block forward substitution.  Here the GPU forms f from g and solves
V_h w = f (the oracle's f) with D_h-preconditioned GMRES in FP64, with the
FP32-stored iterative refinement and, for uniform steps, in block-Toeplitz
storage; w must match element by element.
"""
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
CASES = ["square128_uniform", "lshape48_graded"]


def _load(name):
    path = os.path.join(GOLD, f"solution_{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return np.load(path, allow_pickle=False)


@pytest.mark.parametrize("name", CASES)
def test_solution_matches_oracle(name):
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    z = _load(name)
    c = P.Context(float(z["alpha"]), z["t_nodes"], z["bnd_xy"])
    print("reference solution", name, "N =", c.n, flush=True)
    c.assemble(L.V | L.K | L.D)
    f = c.rhs(z["g"]).cpu().numpy()
    f_ref, w_ref = z["f"], z["w"]
    assert np.linalg.norm(f - f_ref) / np.linalg.norm(f_ref) <= 1e-12
    c.release(L.K)

    def check(w, what):
        w = w.cpu().numpy()
        rel = np.linalg.norm(w - w_ref) / np.linalg.norm(w_ref)
        emax = np.abs(w - w_ref).max() / np.abs(w_ref).max()
        print(name, what, "relative l2", rel, "max", emax, flush=True)
        assert rel <= 1e-10 and emax <= 1e-10, (what, rel, emax)

    w64, i64 = c.solve(f_ref, tol=1e-13, max_it=400)
    check(w64, f"FP64 GMRES ({i64.iters} it)")
    c.release(L.V | L.D)
    c.assemble(L.V | L.D, precision=L.FP32_IR)
    w32, i32 = c.solve(f_ref, tol=1e-13, max_it=400, mode=L.FP32_IR, inner_tol=1e-6, max_outer=12, ir_tol=1e-13)
    check(w32, f"FP32-stored refinement ({i32.outer} outer / {i32.iters} inner)")
    c.release(L.V | L.D)
    h = np.diff(z["t_nodes"])
    if np.abs(h - h[0]).max() <= 1e-12 * h[0]:
        # uniform steps: the block-Toeplitz storage and its matrix-core product
        c.set_toeplitz(True)
        c.assemble(L.V | L.D)
        wt, it = c.solve(f_ref, tol=1e-13, max_it=400)
        check(wt, f"block-Toeplitz FP64 GMRES ({it.iters} it)")
    c.close()
    torch.cuda.empty_cache()
