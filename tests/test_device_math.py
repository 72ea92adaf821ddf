"""The double elementary functions of the double transport path
(paper_2001_11252_amd/csrc/rmc_math.h), built for the host: they are host
and device functions with explicit fmas and contraction off, so these are
the kernels' values.  Their error against 40-digit references (mpmath) stays
under 2 ulp over the arguments the path produces (tan: |th| <= pi/2, edges
and the reduction boundary included; atan: any magnitude; sin and cos of
2 pi r: the uniform draws (2m+1) 2^-53 and the quadrant boundaries; log:
the uniform draws and positive doubles of any magnitude; exp: the
arguments of H(a,x) and of the draw's acceptance test, -x^2 <= 0, and
|x| <= 700), and special arguments give the exact results."""
import ctypes
import os
import subprocess

import mpmath as mp
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("devmath") / "devmath.so")
    p = subprocess.run([HIPCC, "-O2", "-fPIC", "-shared", "-I" + os.path.join(ROOT, "paper_2001_11252_amd", "csrc"),
                        "-o", out, os.path.join(ROOT, "tests", "devmath", "devmath.cpp")],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert p.returncode == 0, p.stdout[-3000:]
    return ctypes.CDLL(out)


def _call(lib, name, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    getattr(lib, name)(x.ctypes.data_as(ctypes.c_void_p), y.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(len(x)))
    return y


def _ulps(y, f, x):
    mp.mp.dps = 40
    out = np.empty(len(x))
    for i, (xi, yi) in enumerate(zip(x, y)):
        r = f(mp.mpf(float(xi)))
        if r == 0:
            out[i] = 0.0 if yi == 0 else np.inf
            continue
        e = int(mp.floor(mp.log(abs(r), 2)))
        out[i] = float(abs(mp.mpf(float(yi)) - r) / mp.mpf(2) ** (e - 52))
    return out


def test_tan_within_2_ulp(lib):
    rng = np.random.default_rng(11)
    hp = np.pi / 2
    th = np.concatenate([rng.uniform(-hp, hp, 4000),
                         hp - np.arange(1, 40) * 2.0 ** -52, -hp + np.arange(1, 40) * 2.0 ** -52,
                         np.pi / 4 + np.arange(-20, 20) * 2.0 ** -53,      # where n changes
                         -np.pi / 4 + np.arange(-20, 20) * 2.0 ** -53,
                         10.0 ** rng.uniform(-300, -1, 200) * rng.choice([-1, 1], 200)])
    y = _call(lib, "devmath_tan_halfpi", th)
    u = _ulps(y, mp.tan, th)
    assert u.max() < 2.0, (u.max(), th[u.argmax()])
    assert u.mean() < 0.5


def test_tan_special_arguments(lib):
    hp = np.pi / 2
    y = _call(lib, "devmath_tan_halfpi", [0.0, -0.0, hp, -hp, 1e-300])
    assert y[0] == 0.0 and y[1] == 0.0 and y[4] == 1e-300
    # tan of the double nearest pi/2 is 1/(pi/2 - that double)
    mp.mp.dps = 40
    ref = float(1 / (mp.pi / 2 - mp.mpf(hp)))
    assert abs(y[2] - ref) <= 2 * np.spacing(ref) and y[3] == -y[2]


def test_atan_within_2_ulp(lib):
    rng = np.random.default_rng(12)
    z = np.concatenate([rng.choice([-1, 1], 4000) * 10.0 ** rng.uniform(-12, 12, 4000),
                        1 + np.arange(-30, 30) * 2.0 ** -52,                    # |z| = 1 switch
                        0.2679491924311227 + np.arange(-30, 30) * 2.0 ** -54,   # tan(pi/12) switch
                        10.0 ** rng.uniform(-300, 300, 200)])
    y = _call(lib, "devmath_atan_any", z)
    u = _ulps(y, mp.atan, z)
    assert u.max() < 2.0, (u.max(), z[u.argmax()])
    assert u.mean() < 0.5


def test_atan_special_arguments(lib):
    y = _call(lib, "devmath_atan_any", [0.0, -0.0, np.inf, -np.inf, 1e-300, 1.0])
    assert y[0] == 0.0 and not np.signbit(y[0]) and y[1] == 0.0 and np.signbit(y[1])
    assert y[2] == np.pi / 2 and y[3] == -np.pi / 2
    assert y[4] == 1e-300
    assert abs(y[5] - np.pi / 4) <= np.spacing(np.pi / 4)


def _uniforms(rng, n):
    # the double path's uniform draws, (2m + 1) 2^-53
    return (2 * rng.integers(0, 2 ** 52, n) + 1) * 2.0 ** -53


def test_sincos_turns_within_2_ulp(lib):
    rng = np.random.default_rng(13)
    r = np.concatenate([_uniforms(rng, 4000), np.arange(1, 9) / 8 + 2.0 ** -53, np.arange(1, 9) / 8 - 2.0 ** -53,
                        [2.0 ** -53, 1 - 2.0 ** -53]])
    s, c = np.empty_like(r), np.empty_like(r)
    lib.devmath_sincos_turns(r.ctypes.data_as(ctypes.c_void_p), s.ctypes.data_as(ctypes.c_void_p),
                             c.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(len(r)))
    us = _ulps(s, lambda v: mp.sinpi(2 * v), r)
    uc = _ulps(c, lambda v: mp.cospi(2 * v), r)
    assert us.max() < 2.0 and uc.max() < 2.0, (us.max(), uc.max())
    # quarter turns are exact
    q = np.arange(0, 9) / 8.0
    s, c = np.empty_like(q), np.empty_like(q)
    lib.devmath_sincos_turns(q.ctypes.data_as(ctypes.c_void_p), s.ctypes.data_as(ctypes.c_void_p),
                             c.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(len(q)))
    assert np.array_equal(s[0::2], [0, 1, 0, -1, 0]) and np.array_equal(c[0::2], [1, 0, -1, 0, 1])


def test_log_within_2_ulp(lib):
    rng = np.random.default_rng(14)
    x = np.concatenate([_uniforms(rng, 4000), 10.0 ** rng.uniform(-300, 300, 1000),
                        1 + np.arange(-40, 40) * 2.0 ** -52, [np.sqrt(0.5), np.nextafter(np.sqrt(0.5), 0), 1e-310,
                                                               5e-324, np.finfo(float).max]])
    y = _call(lib, "devmath_log_pos", x)
    u = _ulps(y, mp.log, x)
    assert u.max() < 2.0, (u.max(), x[u.argmax()])
    assert u.mean() < 0.5
    y = _call(lib, "devmath_log_pos", [1.0, 2.0, 0.5, 2.0 ** -53])
    assert y[0] == 0.0 and y[1] == np.log(2.0) and y[2] == -np.log(2.0)
    assert y[3] == -53 * np.log(2.0) or abs(y[3] + 53 * np.log(2.0)) <= np.spacing(53 * np.log(2.0))


def test_exp_within_2_ulp(lib):
    rng = np.random.default_rng(15)
    x = np.concatenate([-rng.uniform(0, 60, 3000) ** 2 / 60, -10.0 ** rng.uniform(-20, 2.8, 1500),
                        rng.uniform(-700, 700, 1000), np.arange(-20, 20) * np.log(2) / 2])
    y = _call(lib, "devmath_exp_any", x)
    keep = x > -708.0          # normal results
    u = _ulps(y[keep], mp.exp, x[keep])
    assert u.max() < 2.0, (u.max(), x[keep][u.argmax()])
    assert u.mean() < 0.5
    y = _call(lib, "devmath_exp_any", [0.0, -0.0, -746.5, -1e300, 711.0, 1.0, -np.inf])
    assert y[0] == 1.0 and y[1] == 1.0 and y[2] == 0.0 and y[3] == 0.0 and y[4] == np.inf and y[6] == 0.0
    assert abs(y[5] - np.e) <= np.spacing(np.e)
