"""The representation formula (Sec. 1, eq. (2)) at points of Q on the GPU
path (stbem_potential): the three potentials M~0 u0, V~ w and W g.

* parity with the oracle's adaptive long-double potentials, column by
  column, on seeded random data, at points in the middle of Omega, close
  to a side and to a corner, at times on and between the time nodes, small
  and at T;
* u = c0 + c.x is reproduced at interior points (its Cauchy data are exact
  in the discrete spaces), as for the oracle;
* after a solve for the manufactured solution exp(k.x + |k|^2 t / alpha),
  the potentials give u in the interior, with an error that falls on
  refinement;
* points outside Omega or outside (0, T] are rejected."""
import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle

pytestmark = pytest.mark.gpu


def _lshape_small():
    vx, tr = W.lshape_grid(6)
    return W.Workload(name="lshape_small", alpha=0.3, t_nodes=W.graded_times(5, 1.3), bnd_xy=W.lshape_polygon(16),
                      vtx_xy=vx, tri=tr, kvec=np.array([1.0, 0.0]), g=None, u0=None, w_ref=None)


def _points(name, T):
    if name == "tiny":
        xy = [(0.5, 0.5), (0.3, 0.7), (0.999, 0.4), (0.5, 1e-3), (0.001, 0.002), (0.25, 0.5), (0.9, 0.9)]
    else:
        xy = [(0.25, 0.25), (0.7, 0.2), (0.499, 0.75), (0.75, 0.499), (0.4995, 0.5005), (0.1, 0.999), (0.02, 0.3)]
    ts = [T, 0.5 * T, 0.0625, 0.01, 0.3]
    return np.array([(x, y, t) for (x, y) in xy for t in ts])


@pytest.mark.parametrize("name", ["tiny", "lshape_small"])
def test_potentials_match_oracle(name):
    import paper_1811_05224_amd as P
    wl = W.make("tiny") if name == "tiny" else _lshape_small()
    o = Oracle.from_workload(wl)
    c = P.Context.from_workload(wl)
    rng = np.random.default_rng(5)
    w, g, u0 = rng.standard_normal(c.n), rng.standard_normal(c.n), rng.standard_normal(c.nv)
    pts = _points(name, float(wl.t_nodes[-1]))
    got = c.potential(pts, w, g, u0).cpu().numpy()
    ref = o.potential(pts, w, g, u0)
    scale = o.potential(pts, np.abs(w), np.abs(g), np.abs(u0))
    e = np.abs(got - ref) / np.maximum(np.abs(ref), np.abs(scale))
    for col, what in enumerate(("M0~ u0", "V~ w", "W g")):
        i = int(np.argmax(e[:, col]))
        print(name, what, "max error", e[i, col], "at", pts[i], "gpu", got[i, col], "oracle", ref[i, col])
    assert e.max() <= 1e-12
    # without u0 the first column is zero and the others do not change
    got0 = c.potential(pts, w, g).cpu().numpy()
    assert np.all(got0[:, 0] == 0.0) and np.array_equal(got0[:, 1:], got[:, 1:])
    c.close()


def _affine_data(wl, c0, cv):
    bnd = wl.bnd_xy
    d = np.roll(bnd, -1, axis=0) - bnd
    e = d / np.hypot(d[:, 0], d[:, 1])[:, None]
    nrm = np.stack([e[:, 1], -e[:, 0]], 1)
    nt = len(wl.t_nodes) - 1
    return np.tile(nrm @ cv, nt), np.tile(c0 + bnd @ cv, nt), c0 + wl.vtx_xy @ cv


@pytest.mark.parametrize("name", ["tiny", "lshape_small"])
def test_affine_solution_reproduced(name):
    import paper_1811_05224_amd as P
    wl = W.make("tiny") if name == "tiny" else _lshape_small()
    c = P.Context.from_workload(wl)
    c0, cv = 0.7, np.array([0.3, -1.1])
    w, g, u0 = _affine_data(wl, c0, cv)
    pts = _points(name, float(wl.t_nodes[-1]))
    Pt = c.potential(pts, w, g, u0).cpu().numpy()
    u = Pt[:, 0] + Pt[:, 1] - Pt[:, 2]
    err = np.abs(u - (c0 + pts[:, :2] @ cv)).max()
    print(name, "affine solution max error", err)
    assert err <= 1e-12
    c.close()


def test_solve_then_evaluate_converges():
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    pts = np.array([(x, y, t) for (x, y) in [(0.5, 0.5), (0.3, 0.6), (0.8, 0.25)] for t in (0.5, 1.0)])
    errs = []
    for lev in (3, 4, 5):
        n = 2 ** lev
        wl = W.make("custom", n_side=n, n_t=n, n_omega=n, alpha=1.0, k=(0.8, 0.4))
        c = P.Context.from_workload(wl)
        c.assemble(L.V | L.K | L.D | L.M0)
        w, info = c.solve(c.rhs(wl.g, wl.u0), tol=1e-12, max_it=300)
        assert info.status == 0
        Pt = c.potential(pts, w, wl.g, wl.u0).cpu().numpy()
        u = Pt[:, 0] + Pt[:, 1] - Pt[:, 2]
        exact = np.exp(pts[:, :2] @ wl.kvec + (wl.kvec @ wl.kvec) * pts[:, 2] / wl.alpha)
        errs.append(np.abs(u - exact).max() / np.abs(exact).max())
        c.close()
    print("relative max error of u in the interior per level", errs)
    assert errs[-1] <= 1e-2
    assert errs[0] / errs[1] >= 1.8 and errs[1] / errs[2] >= 1.8


def test_points_outside_rejected():
    import paper_1811_05224_amd as P
    wl = W.make("tiny")
    c = P.Context.from_workload(wl)
    w, g = np.zeros(c.n), np.zeros(c.n)
    for bad in ([(1.2, 0.5, 0.5)], [(0.5, 0.5, 0.0)], [(0.5, 0.5, 1.5)], [(0.0, 0.5, 0.5)], [(0.5, 0.5, -0.1)]):
        with pytest.raises(RuntimeError):
            c.potential(bad, w, g)
    assert c.potential(np.zeros((0, 3)), w, g).shape == (0, 3)
    c.close()


def test_points_very_close_to_the_boundary():
    """Points 1e-6 and 1e-9 from a side and from a corner, at a time node and
    between nodes: the graded pieces at the foot of the point keep the
    boundary potentials at the oracle's accuracy (the kernels are nearly
    singular there)."""
    import paper_1811_05224_amd as P
    wl = W.make("tiny")
    o = Oracle.from_workload(wl)
    c = P.Context.from_workload(wl)
    rng = np.random.default_rng(9)
    w, g, u0 = rng.standard_normal(c.n), rng.standard_normal(c.n), rng.standard_normal(c.nv)
    xy = [(0.5, 1e-6), (1e-9, 0.37), (1e-6, 1e-6), (0.999999, 0.5)]
    pts = np.array([(x, y, t) for (x, y) in xy for t in (0.25, 0.3, 1.0)])
    got = c.potential(pts, w, g, u0).cpu().numpy()
    ref = o.potential(pts, w, g, u0)
    scale = o.potential(pts, np.abs(w), np.abs(g), np.abs(u0))
    e = np.abs(got - ref) / np.maximum(np.abs(ref), np.abs(scale))
    print("max error near the boundary per column", e.max(axis=0))
    assert e.max() <= 1e-12
    c.close()
