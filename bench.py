"""Throughput of the weather step on one MI355X.

Workload: the paper's 1581 x 1301 x 58 production grid (2 km, 58 stretched
levels; section "Hybrid ASUCA Strong Scaling GPU Results"), FP32 state,
periodic, seeded synthetic inputs.  One step = three RK3 dycore stages + the
column physics (implicit vertical diffusion with the FP64 fallback, radiation
scan) + the compensated FP64 mass sums, all in the HIP library.

Prints one JSON line:  metric Mcell-steps/s (interior cells x steps / s),
the roofline of the dominant kernel (the RK3 stage kernel) and the FP64 CPU
oracle timed on a bounded sample of the same workload, and the FP32 error
against FP64 after 100 steps on the one-GPU share 400 x 320 x 58.  Unless
--no-surrogate,
the line also carries the learned-physics leg: the MLP surrogate trained on
2,048,000 columns of 400 x 320 x 58 states, its held-out tendency RMSE, and
surrogate and judged steps on the same grid timed against plain steps, with
the MFMA roofline of the inference GEMMs.  Unless --no-reduced it also
carries the paper's reduced weather application (FP64 diffusion + column
physics) at the paper's three benchmark shapes, next to the paper's K20x
times.

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
BF16_PEAK_TFLOPS = 2500.0               # dense BF16 matrix-core peak
# algorithmic network FLOPs per column: 2 (294*512 + 512*512 + 512*116)
MLP_FLOPS_PER_COL = 2 * (294 * 512 + 512 * 512 + 512 * 116)
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


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(budget_s: float = 10.0):
    """The FP64 NumPy oracle on the host, on the 256 x 256 x 58 periodic
    sample of the workload: single-threaded (the whole-grid oracle) and
    threaded (its j-slab driver over the allowed cores, at most 16), each for
    about budget_s seconds; the threaded rate is the reported value."""
    from oracle import dycore, slabs, step
    from paper_1802_05839_amd import inputs

    inp = inputs.generate_config("crop")
    cells = inp.nx * inp.ny * inp.nz
    s = dycore.State(inp.rho.copy(), inp.theta.copy(), inp.q.copy())
    n1 = 0
    t0 = time.perf_counter()
    while True:
        s = step.step(s, inp)
        n1 += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    t1 = time.perf_counter() - t0
    threads = slabs.default_threads()
    slabs.run(inp, 1, threads=threads)          # warm the pool path once
    nt = 0
    t0 = time.perf_counter()
    while True:
        slabs.run(inp, 2, threads=threads)
        nt += 2
        if time.perf_counter() - t0 >= budget_s:
            break
    tt = time.perf_counter() - t0
    single = cells * n1 / t1 / 1e6
    value = cells * nt / tt / 1e6
    return {"value": value, "unit": "Mcell-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"256x256x58 seed-3 grid: {nt} steps in {tt:.1f} s on {threads} threads (the oracle's "
                      f"j-slab driver, bit-identical to the whole-grid oracle); single thread {n1} steps in "
                      f"{t1:.1f} s = {single:.2f} Mcell-steps/s",
            "single_thread_value": round(single, 3), "host_cpu": host_cpu_model(),
            "allowed_cores": slabs.allowed_cores()}


def share_error(steps: int = 100):
    """FP32 against FP64 on the one-GPU share 400 x 320 x 58 after `steps`
    steps of the same library (the FP64 path is pinned to the oracle at
    1e-12): relative L2 and max error per field, theta as theta - 300 K, and
    the mass drift of both runs."""
    import torch

    from paper_1802_05839_amd import inputs, wx

    cfg = inputs.CONFIGS["share"]
    inp = inputs.generate(cfg["nx"], cfg["ny"], cfg["nz"], seed=cfg["seed"])
    i32 = inp.astype(np.float32)
    i32.theta = (inp.theta - 300.0).astype(np.float32).astype(np.float64) + 300.0
    i32.theta_s = (inp.theta_s - 300.0).astype(np.float32).astype(np.float64) + 300.0
    runs = {}
    for name, src, dt, off in (("f64", i32, "f64", 0.0), ("f32", i32, "f32", 300.0)):
        st = wx.state_from_inputs(src, dtype=dt, theta_offset=off)
        m0 = st.mass(compute=True)
        st.step(steps)
        m1 = st.mass()
        f = {k: st.interior(k).double().clone() for k in ("rho", "theta", "q")}
        f["theta"] = f["theta"] + (off - 300.0)
        runs[name] = (f, m0, m1)
        st.close()
    torch.cuda.synchronize()
    out = {"grid": "400x320x58 seed 1", "steps": steps,
           "reference": "FP64 run of the same library (parity-pinned to the oracle at 1e-12)"}
    for k, label in (("rho", "rho"), ("theta", "theta_minus_300"), ("q", "q")):
        a, b = runs["f32"][0][k], runs["f64"][0][k]
        out[label] = {"rel_l2": float(f"{(torch.linalg.norm(a - b) / torch.linalg.norm(b)).item():.3e}"),
                      "rel_max": float(f"{(torch.max(torch.abs(a - b)) / torch.max(torch.abs(b))).item():.3e}")}
    for name in ("f64", "f32"):
        _, m0, m1 = runs[name]
        out[f"mass_drift_{name}"] = [float(f"{x:.3e}") for x in np.abs(m1 - m0) / np.abs(m0)]
    return out


def tendency_rmse(mlp, x_raw, y_raw):
    """Held-out RMSE of the surrogate's tendencies against the plain physics.

    The library normalises the raw feature rows and runs the network
    (wx_mlp_normalize, wx_mlp_infer); the evaluation itself -- undoing the
    target scaling and the RMSE -- is host NumPy in FP64.  Also the
    zero-tendency (no physics) baseline and the training-set std of each
    variable.
    """
    import torch

    from paper_1802_05839_amd import wx

    xn, _ = mlp.normalize(x_raw)
    yn = mlp.infer(xn)
    torch.cuda.synchronize()
    ym = mlp._sec("y_mean", torch.float32, (wx.MLP_NOUTP,)).cpu().numpy().astype(np.float64)
    ys = mlp._sec("y_std", torch.float32, (wx.MLP_NOUTP,)).cpu().numpy().astype(np.float64)
    pred = (yn.cpu().numpy().astype(np.float64) * ys + ym)[:, :wx.MLP_NOUT]
    ref = y_raw[:, :wx.MLP_NOUT].cpu().numpy().astype(np.float64)
    nz = wx.MLP_NZ
    sig = mlp.sigma().cpu().numpy()
    out = {}
    for v, sl in (("theta", slice(0, nz)), ("q", slice(nz, 2 * nz))):
        out[f"rmse_{v}"] = float(np.sqrt(np.mean((pred[:, sl] - ref[:, sl]) ** 2)))
        out[f"rmse_zero_{v}"] = float(np.sqrt(np.mean(ref[:, sl] ** 2)))
    out["sigma_theta"], out["sigma_q"] = float(sig[0]), float(sig[1])
    return out


def surrogate_leg(args, host_inp, stream):
    """Training, held-out RMSE and coupled-step timing of the physics surrogate."""
    import torch

    from paper_1802_05839_amd import surrogate, wx

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    out = {}
    t0 = time.perf_counter()
    x, y = surrogate.build_dataset(log=log)
    torch.cuda.synchronize()
    out["dataset"] = {"rows": int(x.shape[0]),
                      "states": "post-dycore states of steps " + "/".join(map(str, surrogate.SNAPSHOTS))
                                + " of 400x320x58 runs, seeds 100-103",
                      "seconds": round(time.perf_counter() - t0, 2)}
    log(f"dataset {x.shape[0]} rows in {out['dataset']['seconds']} s")
    mlp = wx.Mlp()
    hist, train_s = surrogate.fit(mlp, x, y, epochs=args.train_epochs, batch=4096, lr=1e-3, log=log)
    nsteps = (int(x.shape[0]) // 4096) * args.train_epochs
    del x, y
    torch.cuda.empty_cache()
    held = {}
    for n, (xh, yh) in surrogate.held_out().items():
        rm = tendency_rmse(mlp, xh, yh)
        held[f"step{n}"] = {**{k: float(f"{v:.4e}") for k, v in rm.items()},
                            "rmse_over_sigma_theta": round(rm["rmse_theta"] / rm["sigma_theta"], 4),
                            "rmse_over_sigma_q": round(rm["rmse_q"] / rm["sigma_q"], 4)}
        del xh, yh
    out["train"] = {"epochs": args.train_epochs, "batch": 4096, "adam_steps": nsteps, "lr": 1e-3,
                    "seconds": round(train_s, 2),
                    "samples_per_s": round(nsteps * 4096 / train_s, 1),
                    "TFLOPs": round(3 * MLP_FLOPS_PER_COL * 4096 * nsteps / train_s / 1e12, 1),
                    "loss_first_epoch": round(hist[0], 5), "loss_last_epoch": round(hist[-1], 5)}
    out["held_out"] = {"state": "post-dycore states of a 400x320x58 run, seed 104", "judge_bound_over_sigma": 0.05,
                       **held}
    log(f"trained {nsteps} steps in {train_s:.1f} s; held-out {out['held_out']}")

    # coupled runs on the benchmark grid: plain, judged and unjudged surrogate
    nx, ny, nz = host_inp.nx, host_inp.ny, host_inp.nz
    ncells = nx * ny * nz
    ncol = nx * ny
    steps = args.coupled_steps
    res = {}
    states = {}
    for mode_name, mode in (("plain", wx.WX_PHYS_PLAIN), ("judged", wx.WX_PHYS_JUDGED),
                            ("surrogate", wx.WX_PHYS_SURROGATE)):
        st = wx.state_from_inputs(host_inp, dtype="f32", theta_offset=300.0)
        if mode != wx.WX_PHYS_PLAIN:
            st.attach_mlp(mlp)
        st.set_phys_mode(mode)
        n = steps if mode_name != "surrogate" else max(1, steps // 5)
        rmse = []
        if mode_name == "judged":
            # ten blocks so that the judge's RMSE is sampled along the run;
            # flags count per wx_step call and are summed over the blocks
            blocks = 10
            ms = 0.0
            flags = {}
            for b in range(blocks):
                k = n // blocks + (1 if b < n % blocks else 0)
                ms += timed(lambda: st.step(k))
                rmse.append(st.judge())
                for key, val in st.flags().items():
                    flags[key] = flags.get(key, 0) + val
        else:
            ms = timed(lambda: st.step(n))
            flags = st.flags()
        r = {"steps": n, "ms_per_step": round(ms / n, 4), "Mcell_steps_per_s": round(ncells * n / ms / 1e3, 1),
             "flags": flags}
        if rmse:
            r["judge_rmse_theta"] = [float(f"{j[0]:.3e}") for j in rmse]
            r["judge_rmse_q"] = [float(f"{j[1]:.3e}") for j in rmse]
            r["judge_sampled_columns"] = int(rmse[-1][3])
            r["judge_columns_over_bound_theta"] = [round(j[4], 4) for j in rmse]
            r["judge_columns_over_bound_q"] = [round(j[5], 4) for j in rmse]
            r["fallback_steps"] = flags["fallback_steps"]
        # the state after exactly n steps, before the profiling steps below
        if mode_name in ("plain", "judged"):
            states[mode_name] = {f: st.interior(f).double() for f in ("theta", "q")}
        if mode != wx.WX_PHYS_PLAIN:
            prof = dict(zip(wx.PROFILE_CLASSES, st.profile(min(n, args.profile_steps), stream).tolist()))
            r["per_launch_ms"] = {k: round(v, 4) for k, v in prof.items() if v > 0}
        res[mode_name] = r
        st.close()
        log(f"{mode_name}: {r['ms_per_step']} ms/step")
    # the judged run against the plain run after the same number of steps
    # (theta as stored: the deviation from 300 K)
    div = {}
    for f in ("theta", "q"):
        a = states["judged"][f]
        b = states["plain"][f]
        div[f] = float(f"{(torch.linalg.norm(a - b) / torch.linalg.norm(b)).item():.3e}")
    del states
    res["judged_vs_plain_rel_l2"] = div
    out["coupled"] = res

    # MFMA roofline of the fused surrogate kernel (one launch over all columns:
    # feature rows, three BF16 layers, tendency update)
    prof = res["surrogate"]["per_launch_ms"]
    fused_ms = prof.get("surrogate", 0.0)
    if fused_ms > 0:
        achieved = MLP_FLOPS_PER_COL * ncol / (fused_ms / 1e3) / 1e12
        out["roofline_mlp"] = {"bound": "mfma", "achieved": round(achieved, 1), "peak": BF16_PEAK_TFLOPS,
                               "unit": "TFLOP/s", "frac": round(achieved / BF16_PEAK_TFLOPS, 4),
                               "kernel": "k_surrogate_fused (features + 3 BF16 layers + update)",
                               "launch_ms": round(fused_ms, 4), "flops_per_column": MLP_FLOPS_PER_COL}
    out["speed_vs_plain"] = {k: round(res["plain"]["ms_per_step"] / res[k]["ms_per_step"], 3)
                             for k in ("judged", "surrogate")}
    return out


# the paper's reduced-application timings on a Tesla K20x (FP64, 100 time
# steps, 32 x 16 blocks, host-device copies included; table "Block Size
# Impact on Execution Time" and the appendix on the measurement setup): context
PAPER_RW_K20X_S = {(128, 128, 128): 0.10, (256, 256, 256): 0.55, (256, 256, 512): 2.16}


def reduced_app_leg(stream, steps: int = 100):
    """The paper's reduced weather application (FP64) at its three benchmark shapes."""
    import torch

    from paper_1802_05839_amd import inputs, wx

    res = {}
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    for (nx, ny, nz), k20x_s in PAPER_RW_K20X_S.items():
        e = inputs.rw_box_init(nx, ny, nz)
        surf, pbl = inputs.rw_boundary_fields(nx, ny)
        app = wx.ReducedApp(e, surf, pbl, inputs.RW_NU_DEFAULT)
        app.run(10, stream)
        torch.cuda.synchronize()
        ev0.record(stream)
        app.run(steps, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        # the same run with the field copied in from pinned host memory and
        # back out, as the paper's GPU times include the copies
        host = torch.from_numpy(e).pin_memory()
        back = torch.empty_like(host).pin_memory()
        torch.cuda.synchronize()
        ev0.record(stream)
        app.buf[0].copy_(host, non_blocking=True)
        app.cur = 0
        app.run(steps, stream)
        back.copy_(app.field, non_blocking=True)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_copies = ev0.elapsed_time(ev1)
        cells = nx * ny * nz
        stored = (nx + 2) * (ny + 2) * nz
        gbs = 16 * stored * steps / (ms / 1e3) / 1e9
        # the same run on the KIJ storage order (k fastest), one thread per column
        kij = wx.ReducedApp(e, surf, pbl, inputs.RW_NU_DEFAULT, order="kij")
        kij.run(5, stream)
        torch.cuda.synchronize()
        ev0.record(stream)
        kij.run(steps, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_kij = ev0.elapsed_time(ev1)
        del kij
        res[f"{nx}x{ny}x{nz}"] = {"ms_per_100_steps": round(ms * 100 / steps, 3),
                                  "kij_order_ms_per_100_steps": round(ms_kij * 100 / steps, 3),
                                  "kij_over_ijk": round(ms_kij / ms, 2),
                                  "Mcell_steps_per_s": round(cells * steps / (ms / 1e3) / 1e6, 1),
                                  "algorithmic_GBs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                                  "ms_per_100_steps_with_copies": round(ms_copies * 100 / steps, 3),
                                  "paper_k20x_s_per_100_steps": k20x_s,
                                  "speedup_vs_paper_k20x_with_copies": round(k20x_s * 1e3 / (ms_copies * 100 / steps), 1)}
        del app
        log(f"reduced app {nx}x{ny}x{nz}: {res[f'{nx}x{ny}x{nz}']}")
    # the FP64 oracle for one step at 128^3 on the host, for scale
    from oracle import reduced as rw
    e = inputs.rw_box_init(128, 128, 128)
    surf, pbl = inputs.rw_boundary_fields(128, 128)
    t0 = time.perf_counter()
    rw.step(e, surf, pbl)
    res["oracle_ms_per_step_128"] = round((time.perf_counter() - t0) * 1e3, 1)
    res["paper_k20x_kij_over_ijk_128"] = 7.7     # 0.77 s vs 0.10 s, table "Influence of Storage Order"
    res["note"] = ("FP64, the printed physics-then-diffusion step fused into one kernel (16 algorithmic B per "
                   "stored cell), bit-identical to the oracle; 'with_copies' adds the host-to-device copy of the "
                   "initial field and the copy back from pinned memory, as the paper's K20x times do; those are "
                   "another machine's numbers, context rather than a target")
    return res


def ablation_leg(host_inp, stream, steps: int = 10):
    """Stage-kernel tile shapes and physics-kernel variants on the benchmark
    grid (the MI355X analogue of the paper's block-size table): average launch
    time of each stage and of the physics per variant, from wx_profile_step
    (HIP events on the launch stream).  Every variant gives the same bytes."""
    from paper_1802_05839_amd import wx

    ncells = host_inp.nx * host_inp.ny * host_inp.nz
    out = {"grid": f"{host_inp.nx}x{host_inp.ny}x{host_inp.nz} FP32", "steps_profiled": steps, "stage_tiles": {},
           "physics_kernels": {}}
    shapes = {0: "64x8 (stage 2 on 64x12, the default)", 1: "64x4", 2: "64x12", 3: "32x16", 4: "128x4", 5: "64x8 shared faces"}
    st = wx.state_from_inputs(host_inp, dtype="f32", theta_offset=300.0)
    for tile, name in shapes.items():
        st.set_param("stage_tile", tile)
        st.step(1)
        prof = st.profile(steps, stream).tolist()
        d1, d2, d3 = prof[1:4]
        gbs = sum(VALUES_STAGE.values()) * 4 * ncells / ((d1 + d2 + d3) / 1e3) / 1e9
        out["stage_tiles"][name] = {"stage1_ms": round(d1, 4), "stage2_ms": round(d2, 4), "stage3_ms": round(d3, 4),
                                    "algorithmic_GBs": round(gbs, 1)}
        log(f"stage tile {name}: {out['stage_tiles'][name]}")
    st.set_param("stage_tile", 0)
    for var, name in ((0, "column in registers, 1 wave/SIMD"), (1, "column re-read, 2 waves/SIMD"),
                      (2, "wave per column, lane scans"), (3, "column in registers, 16-byte row loads"),
                      (4, "two lanes per column, two waves/SIMD")):
        st.set_param("phys_kernel", var)
        st.step(1)
        d = st.profile(steps, stream).tolist()[4]
        out["physics_kernels"][name] = {"ms": round(d, 4),
                                        "algorithmic_GBs": round(VALUES_PHYSICS * 4 * ncells / (d / 1e3) / 1e9, 1)}
        log(f"physics kernel {name}: {out['physics_kernels'][name]}")
    st.close()
    return out


def rw_block_leg(stream, steps: int = 100):
    """The reduced application's thread-block sweep at the paper's three
    shapes (its table "Block Size Impact on Execution Time" compares the
    compiler's default 128 x 1 with 32 x 16)."""
    import torch

    from paper_1802_05839_amd import inputs, wx

    res = {}
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    for (nx, ny, nz) in PAPER_RW_K20X_S:
        e = inputs.rw_box_init(nx, ny, nz)
        surf, pbl = inputs.rw_boundary_fields(nx, ny)
        row = {}
        for blk in ((64, 8), (32, 16), (128, 1), (64, 4), (128, 4)):
            app = wx.ReducedApp(e, surf, pbl, inputs.RW_NU_DEFAULT, block=blk)
            app.run(5, stream)
            torch.cuda.synchronize()
            ev0.record(stream)
            app.run(steps, stream)
            ev1.record(stream)
            torch.cuda.synchronize()
            row[f"{blk[0]}x{blk[1]}"] = round(ev0.elapsed_time(ev1) * 100 / steps, 3)
            del app
        res[f"{nx}x{ny}x{nz}"] = {"ms_per_100_steps": row}
        log(f"reduced app blocks {nx}x{ny}x{nz}: {row}")
    res["paper_k20x_s_per_100_steps"] = {"automatic (128x1)": [0.095, 0.63, 2.99], "32x16": [0.10, 0.55, 2.16]}
    return res


# HEVI short step: algorithmic values per cell.  The first stage reads u, v,
# w, b, pi and writes its pi; the second reads the same five and the first
# stage's pi and writes u, v, w, b, pi.
VALUES_HEVI = 6 + 11


def hevi_leg(nx: int, ny: int, nz: int, stream, steps: int = 50):
    """Fast-mode (HEVI) short steps at the benchmark grid, FP32: time per short
    step and the HBM roofline of its two launches, for the two-lane kernel
    (the default), the one-lane register kernel and the one that parks the
    column in its outputs."""
    import torch

    from paper_1802_05839_amd import inputs, wx

    f = inputs.hevi_fields(nx, ny, nz, seed=2).astype(np.float32)
    ncells = nx * ny * nz
    out = {}
    for kernel, name in ((0, "registers"), (1, "parked"), (2, "two_sided")):
        hv = wx.Hevi(f, inputs.HEVI_TAU_DEFAULT, dtype="f32", kernel=kernel)
        hv.run(4, stream)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        hv.run(steps, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        gbs = VALUES_HEVI * 4 * ncells / (ms / 1e3) / 1e9
        del hv
        out[name] = {"ms_per_short_step": round(ms, 4), "Mcell_steps_per_s": round(ncells / (ms / 1e3) / 1e6, 1),
                     "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": round(gbs / HBM_PEAK_GBS, 4)}}
    del f
    return {"workload": f"HEVI short step {nx}x{ny}x{nz} FP32 (two stages, vertical tridiagonal solve per column)",
            "steps": steps, "algorithmic_bytes_per_cell": VALUES_HEVI * 4, **out}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="full", choices=["full", "share", "crop", "tiny"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-share-error", action="store_true")
    ap.add_argument("--train-epochs", type=int, default=120)
    ap.add_argument("--coupled-steps", type=int, default=500)
    ap.add_argument("--no-reduced", action="store_true")
    ap.add_argument("--no-hevi", action="store_true")
    ap.add_argument("--ablation", action="store_true",
                    help="also sweep the stage-kernel tiles, the physics kernels and the reduced application's "
                         "thread blocks")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(no I/J decomposition or halo exchange between GPUs)", file=sys.stderr)
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
    d_halo, d1, d2, d3, d_phys, d_mass = prof.tolist()[:6]
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
    if not args.no_hevi:
        log("HEVI fast-mode short steps")
        out["hevi"] = hevi_leg(nx, ny, nz, stream)
        log(f"hevi: {out['hevi']}")
    if args.ablation:
        out["ablation"] = ablation_leg(inp, stream)
        if not args.no_reduced:
            out["ablation"]["reduced_app_blocks"] = rw_block_leg(stream)
    if not args.no_surrogate and nz == 58:
        out["surrogate"] = surrogate_leg(args, inp, stream)
    if not args.no_reduced:
        out["reduced_app"] = reduced_app_leg(stream)
    if not args.no_share_error:
        log("FP32 against FP64 on the one-GPU share")
        out["fp32_error_share"] = share_error()
    del inp
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
