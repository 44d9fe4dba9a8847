"""Accuracy of the FP64 elementary functions the step kernels use
(paper_2211_12616_amd/csrc/mpt_math.h), compiled for the host from the same
source and compared with extended-precision (x87 long double) references over
the argument ranges the step feeds them:

* ln of a Box-Muller uniform ((k + 1/2) / 2^24, k < 2^24) and of any normal
  number around the reduction boundaries;
* cos of a latitude in degrees, including the poles and a small overshoot
  past them (the midpoint position is not reflected before it is used);
* sin(pi t), cos(pi t) for t = 2u in [0, 2], including every quarter period,
  and cos(pi t) alone by the half-period form;
* the square root of Box-Muller radii (-2 ln u) and of variances, and the
  division inside ln (numerator in [-0.3, 0.42], denominator in [1.7, 2.42]),
  both refined from reciprocal seeds: within 1 ulp.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2211_12616_amd", "csrc")
LD = np.longdouble
PI = LD("3.14159265358979323846264338327950288")


@pytest.fixture(scope="module")
def m64(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    if np.finfo(LD).nmant < 63:
        pytest.skip("no extended-precision long double on this host")
    exe = str(tmp_path_factory.mktemp("m64") / "math64_host")
    subprocess.run([hipcc, "-O2", "-I", CSRC, os.path.join(HERE, "host", "math64_host.cpp"),
                    "-o", exe], check=True, capture_output=True)

    def run(fn, x):
        x = np.ascontiguousarray(x, np.float64)
        out = subprocess.run([exe, fn], input=x.tobytes(), capture_output=True, check=True).stdout
        return np.frombuffer(out, np.float64)
    return run


def ulp_err(got, ref):
    ref64 = ref.astype(np.float64)
    return np.abs(got.astype(LD) - ref) / np.spacing(np.abs(ref64)).astype(LD)


def test_ln_on_box_muller_uniforms(m64):
    rng = np.random.default_rng(5)
    k = np.concatenate([np.arange(0, 4096), (1 << 24) - 1 - np.arange(0, 4096),
                        rng.integers(0, 1 << 24, 400_000)])
    u = (k.astype(np.float64) + 0.5) / 16777216.0
    got = m64("ln", u)
    ref = np.log(u.astype(LD))
    assert ulp_err(got, ref).max() <= 2.0


def test_ln_reduction_boundaries(m64):
    s2 = np.float64(np.sqrt(0.5))
    steps = np.arange(-64, 65)
    m = s2 + steps * np.spacing(s2)
    x = np.concatenate([np.ldexp(m[None, :], np.arange(-1000, 1000, 37)[:, None]).ravel(),
                        np.ldexp(1.0, np.arange(-1020, 1020)),
                        1.0 + np.arange(-64, 65) * np.spacing(1.0)])
    x = x[x > 0]
    got = m64("ln", x)
    ref = np.log(x.astype(LD))
    nz = ref != 0
    assert np.all(got[~nz] == 0.0)
    assert ulp_err(got[nz], ref[nz]).max() <= 2.0


def test_cos_of_latitude(m64):
    rng = np.random.default_rng(6)
    lat = np.concatenate([rng.uniform(-90.0, 90.0, 400_000),
                          [0.0, -0.0, 45.0, -45.0, 90.0, -90.0, 89.999, -89.999, 60.0],
                          90.0 - np.logspace(-12, 0, 200), -90.0 + np.logspace(-12, 0, 200)])
    got = m64("coslat", lat)
    # cos(lat) = sin(90 deg - |lat|) in extended precision (90 - |lat| is
    # exact there); cos of the rounded angle would cancel near the poles
    ref = np.sin((90 - np.abs(lat.astype(LD))) * PI / 180)
    # relative accuracy is kept up to the poles (what 1/cos(lat) needs)
    pole = np.abs(lat) == 90.0
    assert np.all(np.abs(got[pole]) < 1e-16)
    assert ulp_err(got[~pole], ref[~pole]).max() <= 4.0


def test_cos_of_latitude_past_the_pole_is_negative(m64):
    lat = np.concatenate([90.0 + np.logspace(-10, -0.5, 50), -90.0 - np.logspace(-10, -0.5, 50)])
    got = m64("coslat", lat)
    ref = np.cos(lat.astype(LD) * PI / 180)
    assert np.all(got < 0)
    assert np.abs(got - ref.astype(np.float64)).max() < 1e-15


def test_sincospi_on_twice_a_uniform(m64):
    rng = np.random.default_rng(7)
    k = np.concatenate([np.arange(0, 2048), (1 << 24) - 1 - np.arange(0, 2048),
                        rng.integers(0, 1 << 24, 200_000)])
    t = 2.0 * ((k.astype(np.float64) + 0.5) / 16777216.0)
    quarters = np.arange(0, 9) / 4.0
    near = (quarters[:, None] + np.arange(-8, 9)[None, :] * 2.0 ** -25).ravel()
    t = np.concatenate([t, quarters, near[(near >= 0) & (near <= 2)]])
    sc = m64("sincospi", t).reshape(-1, 2)
    # reference by exact half-period reduction: f = t - floor(t),
    # sin(pi t) = +-sin(pi min(f, 1 - f)), cos(pi t) = +-sin(pi (1/2 - f))
    tl = t.astype(LD)
    fl = np.floor(tl)
    f = tl - fl
    sgn = np.where(fl % 2 == 0, LD(1), LD(-1))
    ref_s = sgn * np.sin(PI * np.minimum(f, 1 - f))
    ref_c = sgn * np.sin(PI * (LD(0.5) - f))
    assert np.abs(ref_s - np.sin(PI * tl)).max() < 1e-17          # the reduction itself
    for got, ref in ((sc[:, 0], ref_s), (sc[:, 1], ref_c)):
        assert np.abs(got.astype(LD) - ref).max() <= 2.5e-16         # absolute, as Box-Muller uses it
        big = np.abs(ref) > 1e-8
        assert ulp_err(got[big], ref[big]).max() <= 4.0
    # exact values at t = 0, 1/2, 1, 3/2, 2
    q = sc[len(k):len(k) + 9][0::2]
    np.testing.assert_array_equal(q[:, 0] + 0.0, [0.0, 1.0, 0.0, -1.0, 0.0])
    np.testing.assert_array_equal(q[:, 1] + 0.0, [1.0, 0.0, -1.0, 0.0, 1.0])


def test_cospi_half_period_form(m64):
    # t = 2u for every uniform of the form ((k >> 8) + 1/2) / 2^24 near the
    # ends, the zeros and the extremes of cos(pi t), and a random sample
    rng = np.random.default_rng(10)
    k = np.concatenate([np.arange(0, 4096), (1 << 24) - 1 - np.arange(0, 4096),
                        (1 << 22) + np.arange(-2048, 2048), (3 << 22) + np.arange(-2048, 2048),
                        (1 << 23) + np.arange(-2048, 2048), rng.integers(0, 1 << 24, 400_000)])
    t = 2.0 * ((k.astype(np.float64) + 0.5) / 16777216.0)
    got = m64("cospi", t)
    tl = t.astype(LD)
    fl = np.floor(tl)
    f = tl - fl
    ref = np.where(fl % 2 == 0, LD(1), LD(-1)) * np.sin(PI * (LD(0.5) - f))
    assert np.abs(got.astype(LD) - ref).max() <= 2.5e-16
    big = np.abs(ref) > 1e-8
    assert ulp_err(got[big], ref[big]).max() <= 4.0
    # the same values as the quarter-period form within 2 ulp of 1
    sc = m64("sincospi", t).reshape(-1, 2)
    assert np.abs(got - sc[:, 1]).max() <= 4.5e-16
    np.testing.assert_array_equal(m64("cospi", np.array([0.5, 1.0, 1.5])) + 0.0, [0.0, -1.0, 0.0])


def test_sqrt_on_radii_and_variances(m64):
    rng = np.random.default_rng(8)
    u = (np.arange(1 << 16, dtype=np.float64) * 256 + 0.5) / 2.0 ** 24
    x = np.concatenate([-2.0 * np.log(u), 10.0 ** rng.uniform(-12, 6, 200_000),
                        2.0 ** np.arange(-60.0, 61.0), [1.0, 2.0, 3.0, 4.0, 0.25, 1e-30, 1e30]])
    got = m64("sqrt", x)
    ref = np.sqrt(x.astype(LD))
    assert ulp_err(got, ref).max() <= 1.0


def test_division_in_ln_reduction(m64):
    rng = np.random.default_rng(9)
    m = np.concatenate([rng.uniform(0.70710678118654752440, 1.4142135623730951, 200_000),
                        [0.70710678118654752440, 1.0, 1.4142135623730950]])
    ab = np.empty(2 * len(m))
    ab[0::2] = m - 1.0
    ab[1::2] = m + 1.0
    got = m64("div", ab)
    ref = (m - 1.0).astype(LD) / (m + 1.0).astype(LD)
    nz = ref != 0
    assert ulp_err(got[nz], ref[nz]).max() <= 1.0
    assert np.all(got[~nz] == 0.0)
