"""Writes the oracle regression fixtures in this folder.  Calls only the
oracle and the input generators.

c1_oracle_60steps.json: 32 parcels of the tiny workload (2 deg grid, 30
levels, 2 time levels; particles seed 21) after 60 full steps (advection,
turbulent and mesoscale diffusion, dt = 180 s, Philox key 221112616).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import inputs  # noqa: E402
import oracle  # noqa: E402


def make():
    met = inputs.make_met_c1(seed=11)
    part = inputs.make_particles(10_000, 21).subset(slice(0, 10_000, 313))
    start = part.copy()
    oracle.run(oracle.Met(met), oracle.ctl(), part, 0, 60, nthreads=1)
    return {
        "what": "oracle state after 60 steps, tiny workload, all modules",
        "start": {k: getattr(start, k).tolist() for k in ("lon", "lat", "p", "id")},
        "end": {k: getattr(part, k).tolist() for k in ("lon", "lat", "p", "up", "vp", "wp")},
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "c1_oracle_60steps.json"), "w") as f:
        json.dump(make(), f, indent=1)
