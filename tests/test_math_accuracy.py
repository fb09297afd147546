"""The library's FP64 exponential and logarithm (used by the chemistry's
rate fits) against the C library, in units in the last place, over the
arguments the fits take: T in [1, 1e9] K and the derived powers, and the
exponents down to the underflow threshold."""
import ctypes
import subprocess
from pathlib import Path

import numpy as np
import pytest

ROOT = Path(__file__).resolve().parents[1]


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = tmp_path_factory.mktemp("mathlib") / "libmathcheck.so"
    cmd = ["/opt/rocm/bin/hipcc", "-O2", "-fPIC", "-shared", "-std=c++17", "-ffp-contract=off",
           f"-I{ROOT / 'paper_2404_17630_amd' / 'csrc'}", str(ROOT / "tests" / "math_check.cpp"), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    L = ctypes.CDLL(str(out))
    for f in (L.rt_exp_many, L.rt_log_many):
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_long]
    return L


def call(f, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    f(x.ctypes.data, y.ctypes.data, x.size)
    return y


def ulps(a, b):
    return np.abs(a - b) / np.spacing(np.abs(b))


def test_exp_accuracy(lib):
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-745.0, 709.0, 200000), rng.uniform(-5, 5, 200000),
                        -470000.0 / np.geomspace(1.0, 1e9, 20000), [0.0, 1.0, -1.0, 1e-300, -1e-300]])
    ref = np.exp(x)
    got = call(lib.rt_exp_many, x)
    normal = ref > np.finfo(float).tiny
    assert ulps(got[normal], ref[normal]).max() <= 3
    # results below the normal range keep their absolute accuracy
    assert np.abs(got[~normal] - ref[~normal]).max() <= 2 * np.finfo(float).smallest_subnormal
    assert call(lib.rt_exp_many, np.array([-800.0, 800.0])).tolist() == [0.0, np.inf]


def test_log_accuracy(lib):
    rng = np.random.default_rng(1)
    x = np.concatenate([np.exp(rng.uniform(-700, 700, 200000)), rng.uniform(0.5, 2.0, 200000),
                        np.geomspace(1.0, 1e9, 20000), 1.0 + np.geomspace(1e-15, 1e-3, 1000),
                        [1.0, 2.0, 0.5, np.finfo(float).tiny, 5e-324, 1e308]])
    ref = np.log(x)
    got = call(lib.rt_log_many, x)
    big = np.abs(ref) > 1e-300
    assert ulps(got[big], ref[big]).max() <= 3
    assert np.all(got[x == 1.0] == 0.0)
