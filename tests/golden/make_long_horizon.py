"""Write the long-horizon oracle fixtures ``long_horizon_<config>.npz``.

Calls only the oracle (its j-slab driver, bit-identical to the whole-grid
oracle) and the seeded input generators.  For each configuration the FP64
oracle advances the FP32-representable problem (theta and theta_s rounded
as theta - 300 K, the GPU's stored form) for the stated number of steps and
the fixture keeps, per field (rho, theta - 300 K, q):
  * the values at 4096 cells drawn with numpy's PCG64 seeded 2024 (flat
    indices into the (nz, ny, nx) array, stored with the file);
  * the whole field's L2 norm, max |value|, max and min (the denominators
    of the relative and normalized errors).
Running the oracle over these horizons takes minutes per configuration on a
workstation, far longer than a GPU test may take, hence the fixture.

    python -m tests.golden.make_long_horizon [crop|share ...]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import slabs  # noqa: E402
from paper_1802_05839_amd import inputs  # noqa: E402

CASES = {"crop": 200, "share": 100}
NSAMPLE = 4096
SAMPLE_SEED = 2024


def f32_problem(cfg: str):
    c = inputs.CONFIGS[cfg]
    inp = inputs.generate(c["nx"], c["ny"], c["nz"], seed=c["seed"])
    out = inp.astype(np.float32)
    out.theta = (inp.theta - 300.0).astype(np.float32).astype(np.float64) + 300.0
    out.theta_s = (inp.theta_s - 300.0).astype(np.float32).astype(np.float64) + 300.0
    return out


def sample_index(shape) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    return np.sort(rng.choice(int(np.prod(shape)), size=NSAMPLE, replace=False))


def path(cfg: str) -> str:
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), f"long_horizon_{cfg}.npz")


def make(cfg: str) -> None:
    nsteps = CASES[cfg]
    inp = f32_problem(cfg)
    t0 = time.perf_counter()
    ref = slabs.run(inp, nsteps)
    idx = sample_index(ref.rho.shape)
    out = {"nsteps": np.array(nsteps), "index": idx}
    for name, arr in (("rho", ref.rho), ("theta", ref.theta - 300.0), ("q", ref.q)):
        flat = arr.ravel()
        out[f"{name}_sample"] = flat[idx]
        out[f"{name}_stats"] = np.array([np.linalg.norm(flat), np.max(np.abs(flat)), np.max(flat), np.min(flat)])
    np.savez(path(cfg), **out)
    print(f"{cfg}: {nsteps} steps in {time.perf_counter() - t0:.0f} s -> {path(cfg)}", flush=True)


if __name__ == "__main__":
    for cfg in (sys.argv[1:] or list(CASES)):
        make(cfg)
