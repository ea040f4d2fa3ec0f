"""Throughput of the weather step on one MI355X.

Workload: the paper's 1581 x 1301 x 58 production grid (2 km, 58 stretched
levels; section "Hybrid ASUCA Strong Scaling GPU Results"), FP32 state,
periodic, seeded synthetic inputs.  One step = three RK3 dycore stages + the
column physics (implicit vertical diffusion with the FP64 fallback, radiation
scan) + the compensated FP64 mass sums, all in the HIP library.

Prints one JSON line:  metric Mcell-steps/s (interior cells x steps / s),
the roofline of the dominant kernel (the RK3 stage kernel) and the FP64 CPU
oracle timed on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 200] [--warmup 5] [--config full]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic values moved per interior cell (FP32: 4 B each)
VALUES_STAGE = {1: 9, 2: 12, 3: 12}     # stage input (3) [+ base (3)] + u, v, w + output (3)
VALUES_PHYSICS = 7                      # rho, theta, q, u, v in; theta, q out
COUNTERS_FILE = os.path.join(ROOT, "profiles", "stage_kernel_counters.json")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("k_dycore.hip", "wx_internal.h"):
        with open(os.path.join(ROOT, "paper_1802_05839_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_counters(ncells: int):
    """HBM bytes per stage launch from the committed rocprofv3 counter summary.

    None when the summary is missing or was taken on a different kernel source.
    """
    if not os.path.exists(COUNTERS_FILE):
        return None
    with open(COUNTERS_FILE) as fh:
        c = json.load(fh)
    if c.get("kernel_sha") != kernel_source_hash() or c.get("ncells") != ncells:
        return None
    return c.get("bytes_per_launch")


def cpu_baseline(budget_s: float = 15.0):
    """FP64 NumPy oracle on a 256 x 256 x 58 periodic sample of the workload."""
    from oracle import dycore, step
    from paper_1802_05839_amd import inputs

    inp = inputs.generate_config("crop")
    s = dycore.State(inp.rho.copy(), inp.theta.copy(), inp.q.copy())
    n = 0
    t0 = time.perf_counter()
    while True:
        s = step.step(s, inp)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    t = time.perf_counter() - t0
    cells = inp.nx * inp.ny * inp.nz
    return {"value": cells * n / t / 1e6, "unit": "Mcell-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} steps of the 256x256x58 seed-3 grid (NumPy FP64, single thread), "
                      f"{t:.1f} s"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="full", choices=["full", "share", "crop", "tiny"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the I/J decomposition is described in DESIGN.md)", file=sys.stderr)
        return 2

    import torch

    from paper_1802_05839_amd import inputs, wx

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    cfg = inputs.CONFIGS[args.config]
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    t0 = time.perf_counter()
    inp = inputs.generate(nx, ny, nz, seed=cfg["seed"], dtype=np.float32)
    log(f"generated {nx}x{ny}x{nz} in {time.perf_counter() - t0:.1f} s, dt={inp.dt:.4f}")
    st = wx.state_from_inputs(inp, dtype="f32", theta_offset=300.0)
    del inp
    torch.cuda.synchronize()
    log("uploaded")
    stream = torch.cuda.current_stream()
    st.step(args.warmup)
    torch.cuda.synchronize()
    log("warmup done")

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    st.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    ms_per_step = ms / args.steps
    ncells = nx * ny * nz
    value = ncells * args.steps / (ms / 1e3) / 1e6
    flags = st.flags()
    mass = st.mass()
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {value:.1f} Mcell-steps/s, flags {flags}")

    # per-kernel durations with HIP events on the same stream
    prof = st.profile(args.profile_steps, stream)
    d_halo, d1, d2, d3, d_phys, d_mass = prof.tolist()
    stage_bytes = sum(VALUES_STAGE.values()) * 4 * ncells
    stage_ms = d1 + d2 + d3
    achieved = stage_bytes / (stage_ms / 1e3) / 1e9
    traffic = traffic_from_counters(ncells)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_stage (RK3 stage, 3 launches per step)",
                "per_launch_ms": {"stage1": round(d1, 4), "stage2": round(d2, 4), "stage3": round(d3, 4),
                                  "physics": round(d_phys, 4), "mass_final": round(d_mass, 4)},
                "physics_GBs": round(VALUES_PHYSICS * 4 * ncells / (d_phys / 1e3) / 1e9, 1)
                if d_phys > 0 else None}
    step_bytes = (sum(VALUES_STAGE.values()) + VALUES_PHYSICS) * 4 * ncells

    # plain copy kernel of the same size as one field: the achievable ceiling
    nbytes = st.field_elems * 4
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    wx.copy_probe(dst, src)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(10):
        wx.copy_probe(dst, src)
    ev1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * nbytes * 10 / (ev0.elapsed_time(ev1) / 1e3) / 1e9
    del src, dst
    st.close()

    out = {
        "metric": "Mcell-steps/s",
        "value": round(value, 1),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"plain-physics weather step {nx}x{ny}x{nz} FP32 "
                               "(RK3 advection + biharmonic + Thomas/FP64-fallback + radiation scan + FP64 mass sums)",
                   "nx": nx, "ny": ny, "nz": nz, "seed": cfg["seed"], "dx_m": 2000.0},
        "hbm_frac_step": round(step_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "algorithmic_bytes_per_cell_step": (sum(VALUES_STAGE.values()) + VALUES_PHYSICS) * 4,
        "copy_kernel_GBs": round(copy_gbs, 1),
        "roofline": roofline,
        "flags": flags,
        "mass": [float(x) for x in mass],
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
