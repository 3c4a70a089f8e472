"""The kernels' special functions, built for the host from the same header
(csrc/stbem_math.h is __host__ __device__), against SciPy and NumPy:
E1 on its three branches (Ein series for z <= 2, half-octave polynomials on
[2, 64), continued fraction beyond), Ein, and the table-driven exponential
of the separated-block tiles.  The bound 4e-15 on z <= 2 comes from
-gamma - ln z + Ein(z) near its smallest value; elsewhere a few ulp."""
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
