"""The natural logarithms the device rate coefficients use (ln T and
ln(1 + u) of the App. E fits), compiled from the same header for the host:
their error in units in the last place against extended precision over the
ranges the chemistry reaches and beyond, and the special arguments.  The
header uses explicit fma() and nothing the compiler may contract, so the
host build computes the same bits as the device build."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "paper_1304_7126_amd", "csrc")

DRIVER = r"""
#include "rt_math.h"
extern "C" void rm_eval(int fn, const double *x, double *y, long n)
{
    for (long i = 0; i < n; ++i) y[i] = fn == 0 ? rtm1::rt_log(x[i]) : rtm1::rt_log1p(x[i]);
}
"""


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("rate_math")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    so = d / "drv.so"
    subprocess.run([cxx, "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-D__host__=",
                    "-D__device__=", "-D__forceinline__=inline", "-I", HEADER_DIR, str(src), "-o", str(so)],
                   check=True)
    return ctypes.CDLL(str(so))


def run(lib, fn, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    lib.rm_eval(fn, x.ctypes.data_as(ctypes.c_void_p), y.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(x.size))
    return y


def ulps(y, ref):
    u = np.spacing(np.abs(ref.astype(np.float64))).astype(np.longdouble)
    return np.abs((y.astype(np.longdouble) - ref) / u).astype(np.float64)


def test_log_accuracy(lib):
    rng = np.random.default_rng(11)
    x = np.concatenate([np.exp(rng.uniform(np.log(1e-300), np.log(1e300), 400_000)),
                        10.0 ** rng.uniform(0, 10, 300_000),        # temperatures
                        rng.uniform(0.5, 2.0, 300_000),             # around the reduction's split
                        rng.uniform(0.999, 1.001, 100_000)])
    x = x[x != 1.0]
    e = ulps(run(lib, 0, x), np.log(x.astype(np.longdouble)))
    assert e.max() < 1.25, (e.max(), x[e.argmax()])
    assert e.mean() < 0.25


def test_log1p_accuracy(lib):
    rng = np.random.default_rng(12)
    u = np.concatenate([10.0 ** rng.uniform(-20, 8, 400_000), rng.uniform(0.0, 3.0, 300_000),
                        10.0 ** rng.uniform(-2, 2, 300_000)])  # (lambda/lambda_0)^q over 10 K .. 1e9 K
    e = ulps(run(lib, 1, u), np.log1p(u.astype(np.longdouble)))
    assert e.max() < 1.6, (e.max(), u[e.argmax()])
    assert e.mean() < 0.35


def test_exact_and_special_arguments(lib):
    assert run(lib, 0, np.array([1.0]))[0] == 0.0
    p2 = 2.0 ** np.arange(-1074, 1024, dtype=np.float64)
    e = ulps(run(lib, 0, p2[p2 != 1.0]), np.log(p2[p2 != 1.0].astype(np.longdouble)))
    assert e.max() < 0.51  # k ln 2 with the split constant: rounded once
    y = run(lib, 0, np.array([0.0, -0.0, -1.0, np.inf, np.nan, 5e-324]))
    assert y[0] == -np.inf and y[1] == -np.inf and np.isnan(y[2]) and y[3] == np.inf and np.isnan(y[4])
    assert y[5] == pytest.approx(np.log(5e-324), rel=1e-15)
    z = run(lib, 1, np.array([0.0, 1e-30, 2.0 ** -53, np.inf, 1e300, np.nan]))
    assert z[0] == 0.0 and z[1] == 1e-30 and z[2] == 2.0 ** -53 and z[3] == np.inf
    assert z[4] == pytest.approx(np.log(1e300), rel=1e-15)
    assert np.isnan(z[5])


def test_monotone_over_temperatures(lib):
    # the rates' logarithmic derivatives rely on a log that does not step
    # backwards between neighbouring arguments
    x = np.nextafter(np.linspace(1.0, 4.0, 200_001), np.inf)
    y = run(lib, 0, x)
    assert np.all(np.diff(y) >= 0.0)
