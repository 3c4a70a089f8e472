"""The kernels' special functions, built for the host from the same header
(csrc/stbem_math.h is __host__ __device__), against SciPy and NumPy:
E1 on its three branches (Ein series for z <= 2, half-octave polynomials on
[2, 64), continued fraction beyond), Ein, and the table-driven exponential
of the separated-block tiles; and the time integrals of separated (series)
and touching (closed forms) blocks against mpmath quadrature.  The E1
bound 4e-15 on z <= 2 comes from -gamma - ln z + Ein(z) near its smallest
value; elsewhere a few ulp."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy.special import exp1

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1811_05224_amd", "csrc")


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("devmath") / "device_math_host")
    subprocess.run([hipcc, "-O2", "-std=c++17", "-I", CSRC, os.path.join(HERE, "device_math_host.cpp"), "-o", exe],
                   check=True, capture_output=True, timeout=600)
    return exe


def run(exe, z):
    out = subprocess.run([exe], input="\n".join(repr(float(v)) for v in z), capture_output=True, text=True,
                         check=True).stdout.split()
    return np.array(out, dtype=np.float64).reshape(-1, 5)


def test_e1_branches_and_exp(prog):
    rng = np.random.default_rng(7)
    z = np.concatenate([10 ** rng.uniform(-8, np.log10(2.0), 400), [2.0, 3.0, 4.0, 6.0, 8.0, 12.0, 16.0, 24.0, 32.0, 48.0],
                        rng.uniform(2, 64, 1200), rng.uniform(64, 700, 300), [np.nextafter(2.0, 3.0), np.nextafter(64.0, 0.0), 64.0]])
    r = run(prog, z)
    e1, ex = r[:, 1], r[:, 2]
    ref = exp1(z)
    rel = np.abs(e1 - ref) / ref
    small = z <= 2.0
    assert rel[small].max() < 4e-15, rel[small].max()
    assert rel[~small].max() < 6e-16, rel[~small].max()
    assert np.abs(ex / np.exp(-z) - 1).max() < 3e-16


def test_ein_and_table_exponential(prog):
    rng = np.random.default_rng(8)
    z = np.concatenate([[0.0, 1e-300, 1e-12, 0.0054, 0.5, 1.0, 2.0], rng.uniform(0, 2, 500)])
    r = run(prog, z)
    # Ein(z) = E1(z) + gamma + ln z; its series is exact at 0
    ein = r[:, 3]
    pos = z > 1e-3
    ref = exp1(z[pos]) + np.euler_gamma + np.log(z[pos])
    assert np.abs(ein[pos] - ref).max() / np.abs(ref).max() < 4e-15
    assert ein[0] == 0.0
    zz = np.concatenate([z, rng.uniform(0, 50, 2000), rng.uniform(50, 740, 200), [745.2, 800.0, 1e6, 1e300]])
    e = run(prog, zz)[:, 4]
    ref = np.exp(-zz)
    big = ref < 1e-300
    assert np.all(e[big] < 1e-300)
    assert (np.abs(e[~big] - ref[~big]) / ref[~big]).max() < 4e-16


def _lag_integral(kern, t, a):
    """int over s of w(s) kern(s, a), w the overlap length of [t2, t3] and
    [t0, t1] + s (the two time elements at lag s), by mpmath."""
    import mpmath as mp
    t0, t1, t2, t3 = (mp.mpf(float(v)) for v in t)
    w = lambda s: max(mp.mpf(0), min(t3, t1 + s) - max(t2, t0 + s))
    br = sorted({t2 - t1, t2 - t0, t3 - t1, t3 - t0})
    return mp.quad(lambda s: w(s) * kern(s, mp.mpf(float(a))), br)


def test_separated_block_series(prog):
    """The series of separated time elements (Laguerre expansion about the
    centre lag, truncated at kSeriesTol) against mpmath quadrature of the
    five lag kernels with the trapezoid weight: equal steps at lags 2, 3, 5,
    12 and 60, and unequal steps, for z = a / dc from 0 to 40.  Bar: 2e-15 of
    the integral of |kernel| times e^{z/2} (the bound of e^{-z} L_n(z) that
    also bounds the truncated tail).  Rounding sets the worst case (8.8e-16,
    the same with the series cut at 1e-19); cut at 1e-13 it fails."""
    import mpmath as mp
    mp.mp.dps = 30
    pi4 = 4 * mp.pi
    kern = [lambda s, a: mp.exp(-a / s) / (pi4 * s),                  # Delta F_V
            lambda s, a: a * mp.exp(-a / s) / s ** 2,                  # Delta F_K
            lambda s, a: mp.exp(-a / s) * (a - s) / (pi4 * s ** 3),    # Delta F_D
            lambda s, a: -mp.exp(-a / s) / (pi4 * s ** 2),             # d/da Delta F_V
            lambda s, a: mp.exp(-a / s) / (pi4 * s ** 3)]              # d2/da2 Delta F_V
    h = 1.0 / 256
    blocks = [(0.0, h, d * h, (d + 1) * h) for d in (2, 3, 5, 12, 60)]
    blocks += [(0.1, 0.14, 0.22, 0.24), (0.1, 0.11, 0.15, 0.17), (0.0, 0.02, 0.5, 0.53)]
    cases = []
    for t in blocks:
        dc = 0.5 * (t[2] + t[3]) - 0.5 * (t[0] + t[1])
        for z in (0.0, 1e-6, 0.3, 1.0, 2.5, 6.0, 15.0, 40.0):
            cases.append((t, z * dc))
    inp = "\n".join(" ".join(repr(float(v)) for v in (*t, a)) for t, a in cases)
    out = subprocess.run([prog, "series"], input=inp, capture_output=True, text=True, check=True).stdout.split()
    got = np.array(out, dtype=np.float64).reshape(-1, 6)
    assert np.all(np.isfinite(got[:, :5])) and np.all(got[:, 5] >= 2)
    worst = 0.0
    for (t, a), row in zip(cases, got):
        dc = 0.5 * (t[2] + t[3]) - 0.5 * (t[0] + t[1])
        grow = float(mp.exp(a / dc / 2))
        for q in range(5):
            ref = _lag_integral(kern[q], t, a)
            scale = _lag_integral(lambda s, aa: abs(kern[q](s, aa)), t, a) * grow
            if scale == 0:
                assert row[q] == 0.0
                continue
            err = float(abs(mp.mpf(row[q]) - ref) / scale)
            worst = max(worst, err)
            assert err <= 2e-15, (t, a, q, err)
    print("worst scaled error", worst)


def test_touching_block_closed_forms(prog):
    """The closed forms of touching time elements (four-point differences of
    the antiderivatives, E1 on its three branches) against mpmath quadrature
    of the lag kernels with the trapezoid weight: an element with itself and
    two adjacent elements of equal and unequal length, z = a / h from 1e-3 to
    60.  Bar: 1e-13 of the integral of |kernel|, with the floor of the
    parity tests (1e-8 of the largest such integral over the block's z):
    the differences cancel by about z^2 where e^{-z} is far below that floor
    (2.4e-13 of the value at z = 60)."""
    import mpmath as mp
    mp.mp.dps = 50
    pi4 = 4 * mp.pi
    kern = [lambda s, a: mp.exp(-a / s) / (pi4 * s),                  # Delta F_V
            lambda s, a: a * mp.exp(-a / s) / s ** 2,                  # Delta F_K
            lambda s, a: mp.exp(-a / s) * (a - s) / (pi4 * s ** 3),    # Delta F_D
            lambda s, a: -a * mp.exp(-a / s) / (pi4 * s ** 2),         # d/dalpha Delta F_V, alpha = 1
            lambda s, a: mp.exp(-a / s) * (a - s) / s ** 3]            # four-point sum of E1
    blocks = [(0, 0.3, 0.32, 0.0), (1, 0.3, 0.32, 0.34), (1, 0.3, 0.31, 0.34)]
    zs = (1e-3, 0.05, 0.5, 1.0, 2.5, 8.0, 30.0, 60.0)
    cases = [(d, t0, t1, t2, z * (t1 - t0)) for d, t0, t1, t2 in blocks for z in zs]
    inp = "\n".join("%d %r %r %r %r" % c for c in cases)
    out = subprocess.run([prog, "touch"], input=inp, capture_output=True, text=True, check=True).stdout.split()
    got = np.array(out, dtype=np.float64).reshape(-1, 5)
    res = []
    for (d, t0, t1, t2, a), row in zip(cases, got):
        m0, m1 = mp.mpf(t0), mp.mpf(t1)
        k0, k1 = (m0, m1) if d == 0 else (mp.mpf(t1), mp.mpf(t2))
        am = mp.mpf(a)
        w = lambda s: max(mp.mpf(0), min(k1, m1 + s) - max(k0, m0 + s))
        corners = [v for v in (k0 - m1, k0 - m0, k1 - m1, k1 - m0) if v > 0]
        # e^{-a/s} piles the integrand up against the largest lags when a is
        # large: points graded toward every corner keep the quadrature exact
        br = sorted({mp.mpf(0), am, 4 * am, *corners, *(c * (1 - mp.mpf(2) ** -j) for c in corners for j in range(1, 12))})
        for q in range(5):
            ref = mp.quad(lambda s: w(s) * kern[q](s, am), br)
            scale = mp.quad(lambda s: w(s) * abs(kern[q](s, am)), br)
            res.append(((d, t0, t1, t2), q, a, float(abs(mp.mpf(row[q]) - ref)), float(scale)))
    top = {}
    for blk, q, a, err, scale in res:
        top[blk, q] = max(top.get((blk, q), 0.0), scale)
    worst = 0.0
    for blk, q, a, err, scale in res:
        rel = err / max(scale, 1e-8 * top[blk, q])
        worst = max(worst, rel)
        assert rel <= 1e-13, (blk, q, a, rel)
    print("worst scaled error", worst)
