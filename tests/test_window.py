"""The launch limit of the R16 step kernels (paper_2211_12616_amd/csrc/
mpt_window.h), compiled for the host.  The kernels keep the per-level scales
of three consecutive met levels in LDS, from the earlier level of the
launch's first time; that is enough only if the earlier level of every time
the launch reads moves by at most one.  Checked here with times formed as
the step forms them (t = t_start + step dt, the last one t + dt/2) and the
level as the step locates it (floor((t - t_met0) / dt_met)), for the longest
launch the limit allows, over many starts, and at the limit's edges: it is
the longest launch that fits, and none fits when half a step exceeds a met
interval."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2211_12616_amd", "csrc")


@pytest.fixture(scope="module")
def limit(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("win") / "window_host")
    subprocess.run([cxx, "-O2", "-std=c++17", "-I", CSRC, os.path.join(HERE, "host", "window_host.cpp"),
                    "-o", exe], check=True, capture_output=True)

    def run(dt, dt_met):
        x = np.ascontiguousarray(np.stack([np.asarray(dt, np.float64), np.asarray(dt_met, np.float64)], 1))
        out = subprocess.run([exe], input=x.tobytes(), capture_output=True, check=True).stdout
        y = np.frombuffer(out, np.float64).reshape(-1, 3)
        return y[:, 0].astype(np.int64), y[:, 1] == 1.0, y[:, 2] == 1.0
    return run


def test_longest_launch_that_fits(limit):
    dt_met = np.array([21600.0, 3600.0, 10800.0, 21600.0, 21600.0, 3600.0, 100.0, 21600.0])
    dt = np.array([180.0, 180.0, 60.0, 21600.0, 43000.0, 7190.0, 0.001, 180.0 * 120 / 119.5])
    n, fits_n, fits_next = limit(dt, dt_met)
    assert np.all(fits_n == (n >= 1))
    assert not np.any(fits_next & (n < 1_000_000_000))
    np.testing.assert_array_equal(n[:3], [120, 20, 180])        # (n - 1/2) dt <= 0.999 dt_met
    assert n[3] == 1 and n[4] == 1 and n[5] == 1                  # half a step inside an interval
    assert n[7] == 119                                            # just past 120


def test_no_launch_when_half_a_step_exceeds_an_interval(limit):
    dt_met = np.full(4, 3600.0)
    dt = np.array([2.0 * 3600.0, 1.999 * 3600.0, 1.998 * 3600.0, 1.99 * 3600.0])
    n, _, _ = limit(dt, dt_met)
    np.testing.assert_array_equal(n, [0, 0, 1, 1])


@pytest.mark.parametrize("dt, dt_met, t_met0", [(180.0, 21600.0, 0.0), (180.0, 3600.0, -1234.5),
                                                (37.0, 3600.0, 7.25), (900.0, 10800.0, 1e6),
                                                (7000.0, 3600.0, 0.0)])
def test_earlier_level_moves_at_most_one(limit, dt, dt_met, t_met0):
    n = int(limit([dt], [dt_met])[0][0])
    assert n >= 1
    rng = np.random.default_rng(5)
    t_start = t_met0 + rng.uniform(-3.0, 3.0, 20000) * dt_met
    step0 = rng.integers(0, 100_000, 20000).astype(np.float64)
    inv = 1.0 / dt_met
    t_first = t_start + step0 * dt
    t_last = (t_start + (step0 + (n - 1)) * dt) + 0.5 * dt
    lev0 = np.floor((t_first - t_met0) * inv)
    lev1 = np.floor((t_last - t_met0) * inv)
    assert np.all(lev1 - lev0 <= 1)
