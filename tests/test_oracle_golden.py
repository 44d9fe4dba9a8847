"""Regression fixture of the oracle (written by tests/golden/make_golden.py,
which calls only the oracle): a change to the oracle's arithmetic shows up
here and must name the passage that justifies it."""
import json
import os

import numpy as np

import inputs
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def test_c1_regression_fixture(met_c1):
    with open(os.path.join(HERE, "golden", "c1_oracle_60steps.json")) as f:
        g = json.load(f)
    part = inputs.make_particles(10_000, 21).subset(slice(0, 10_000, 313))
    np.testing.assert_array_equal(part.lon, g["start"]["lon"])
    oracle.run(oracle.Met(met_c1), oracle.ctl(), part, 0, 60, nthreads=1)
    for k in ("lon", "lat", "p", "up", "vp", "wp"):
        np.testing.assert_allclose(getattr(part, k), g["end"][k], rtol=1e-12, atol=1e-12)
