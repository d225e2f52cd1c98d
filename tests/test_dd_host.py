"""The library's double-double arithmetic (csrc/dd.h, used by the
double-double plain path) built for the host and checked against 60-digit
values: the error-free sum, product and divisions, and the elementary
functions written for it (exp, log, pow, Gamma, sin/cos).  Bounds are about
ten times the measured worst case over the seeded samples; a double-rounded
intermediate (1e-16) anywhere fails them by many orders of magnitude."""
import ctypes
import os
import shutil
import subprocess

import mpmath as mp
import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1710_01133_amd", "csrc")
D2 = ctypes.c_double * 2


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("ddhost") / "libddhost.so")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-fPIC", "-shared",
                    "-std=c++17", "-ffp-contract=off", "-I", CSRC,
                    os.path.join(HERE, "dd_host_shim.hip"), "-o", out],
                   check=True, capture_output=True)
    return ctypes.CDLL(out)


def pair(v):
    hi = float(v)
    return D2(hi, float(v - mp.mpf(hi)))


def val(o):
    return mp.mpf(o[0]) + mp.mpf(o[1])


def rand_dd(rng):
    """A pair whose low part is populated: mantissa perturbed at 2^-60."""
    m = mp.mpf(rng.uniform(-1, 1)) * (1 + mp.mpf(rng.uniform(0, 1)) * mp.mpf(2) ** -60)
    return m * mp.mpf(2) ** int(rng.integers(-20, 20))


def test_sum_product_and_divisions(lib):
    mp.mp.dps = 60
    rng = np.random.default_rng(5)
    worst = {"add": 0.0, "mul": 0.0, "div": 0.0, "div_d": 0.0}
    o = (ctypes.c_double * 2)()
    for _ in range(2000):
        x, y = pair(rand_dd(rng)), pair(rand_dd(rng))
        xv, yv = val(x), val(y)
        lib.t_add(x, y, o)
        worst["add"] = max(worst["add"], float(abs(val(o) - (xv + yv)) / max(abs(xv), abs(yv))))
        lib.t_mul(x, y, o)
        worst["mul"] = max(worst["mul"], float(abs(val(o) - xv * yv) / abs(xv * yv)))
        lib.t_div(x, y, o)
        worst["div"] = max(worst["div"], float(abs(val(o) - xv / yv) / abs(xv / yv)))
        d = float(rng.uniform(1, 1000)) * (1 if rng.uniform() < 0.5 else -1)
        lib.t_div_d(x, ctypes.c_double(d), o)
        worst["div_d"] = max(worst["div_d"], float(abs(val(o) - xv / d) / abs(xv / d)))
    print(worst)
    for k, v in worst.items():
        assert v <= 2.0 ** -103, (k, v)


def test_exp_log_pow(lib):
    mp.mp.dps = 60
    rng = np.random.default_rng(6)
    o = (ctypes.c_double * 2)()
    worst = [0.0, 0.0, 0.0]
    for xv in np.concatenate([rng.uniform(-40, 40, 200), [0.0, 1e-20, 1.0, -1.0, 700.0]]):
        x = pair(mp.mpf(xv))
        lib.t_exp(x, o)
        worst[0] = max(worst[0], float(abs(val(o) - mp.exp(val(x))) / mp.exp(val(x))))
    for xv in np.concatenate([np.exp(rng.uniform(-30, 30, 200)), [1.0 + 2.0 ** -40, 2.0, 199999.0]]):
        x = pair(mp.mpf(xv))
        lib.t_log(x, o)
        ref = mp.log(val(x))
        worst[1] = max(worst[1], float(abs(val(o) - ref) / max(abs(ref), 1)))
    for xv in np.concatenate([rng.uniform(1, 3e5, 100), [2.0, 3.0]]):
        for a in (0.3, 0.55, 0.9, 0.95, 1.5, 2.0):
            x = pair(mp.mpf(xv))
            lib.t_pow(x, ctypes.c_double(a), o)
            ref = val(x) ** mp.mpf(a)
            worst[2] = max(worst[2], float(abs(val(o) - ref) / ref))
    print("exp %.3g log %.3g pow %.3g" % tuple(worst))
    assert worst[0] <= 1e-29     # |x| <= 700: the argument's own rounding is 700 x 2^-106
    assert worst[1] <= 1e-31
    assert worst[2] <= 1e-29


def test_gamma(lib):
    mp.mp.dps = 60
    rng = np.random.default_rng(7)
    o = (ctypes.c_double * 2)()
    worst = 0.0
    for zv in np.concatenate([rng.uniform(0.5, 60, 100), [1.0, 1.9, 2.0, 2.95, 3.0]]):
        z = pair(mp.mpf(zv))
        lib.t_gamma(z, o)
        ref = mp.gamma(val(z))
        worst = max(worst, float(abs(val(o) - ref) / ref))
    print("gamma %.3g" % worst)
    assert worst <= 2e-28


def test_sincos(lib):
    """Absolute error within 1e-31 (|x| + 1): the reduction by a double-double
    pi/2 carries |x| 2^-107 into the reduced argument."""
    mp.mp.dps = 60
    rng = np.random.default_rng(8)
    o = (ctypes.c_double * 4)()
    worst = 0.0
    for xv in np.concatenate([rng.uniform(-300, 300, 300),
                              [0.0, 1e-3, np.pi / 4, np.pi / 2, np.pi, 240.0]]):
        x = pair(mp.mpf(xv))
        lib.t_sincos(x, o)
        xx = val(x)
        e = max(abs(mp.mpf(o[0]) + mp.mpf(o[1]) - mp.sin(xx)),
                abs(mp.mpf(o[2]) + mp.mpf(o[3]) - mp.cos(xx)))
        worst = max(worst, float(e / (abs(xx) + 1)))
    print("sin/cos %.3g of (|x| + 1)" % worst)
    assert worst <= 1e-31
