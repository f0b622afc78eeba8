"""Benchmark: Yee cell-updates/s of the batched FP32 force solve, force-solve
latency percentiles, and the plain one-channel-at-a-time path beside it.

One step = one complete force solve of the 2D TE+TM piston at 400 x 200
(res 40, h = 0.5, 40 cosine harmonics per face clamped to the face's sample
count -> 448 channels, T = 10000 time steps, sigma = 1, Courant 0.5): every
channel is kicked, advanced T steps and its surface correlation integrated
against K(t); the force is reduced on the host.  Inputs (material grids,
tables) are uploaded inside each solve; the timed work is the whole solve.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-plain]

Prints one JSON line.  Only one GPU is used; --gpus > 1 is refused.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Yee cell-updates/s + force-solve p50/p99 latency, batched FP32 vs plain"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(wl, n_channels=16, n_steps=3000):
    """The FP64 oracle as it stands, on a bounded sample of the workload:
    n_channels channels (spread over kinds, faces and polarizations) for
    n_steps steps, one process per channel on the host cores."""
    import oracle
    from oracle.force import setup
    _, _, _, _, chans = setup(wl)
    pick = np.linspace(0, len(chans) - 1, n_channels).astype(int).tolist()
    workers = min(len(pick), os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    oracle.solve(wl, n_steps=n_steps, channel_subset=pick, workers=workers, chunk=1)
    dt = time.perf_counter() - t0
    cu = len(pick) * wl.n_cells * n_steps
    return {"value": cu / dt, "unit": "cell-updates/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(pick)} of {len(chans)} channels x {n_steps} of {wl.n_steps} steps "
                      f"({cu:.3e} cell-updates, {dt:.1f} s, FP64 NumPy, one process per channel)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--n-steps", type=int, default=None, help="override T (testing only)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB (a plain copy kernel of known size, "
                         "the reference for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the channel-parallel "
              "multi-GPU design is described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_0906_5170_amd as cf
    from casimir_inputs import c2_piston_tetm_fp32

    cpu = None
    if not args.no_cpu:
        # before any GPU call: the oracle forks one process per sampled channel
        log("[bench] cpu baseline (oracle) ...")
        cpu = cpu_baseline(c2_piston_tetm_fp32())
        log(f"[bench] cpu baseline {cpu['value']:.3e} cell-updates/s on {cpu['cores']} cores")
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    cf.load()
    wl = c2_piston_tetm_fp32()
    if args.n_steps:
        wl = wl.replace(n_steps=args.n_steps)
    if args.calib_copy_mib:
        n = args.calib_copy_mib * 2**20 // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calib_copy_mib} MiB done")
        del a, b
    prob = cf.Problem.from_workload(wl)
    opts = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol=wl.pol,
                kernel=wl.kernel, precision="fp32")
    info = prob.info(**opts)
    ws = torch.empty(info["workspace_bytes"], dtype=torch.uint8, device="cuda")
    log(f"[bench] {wl.name}: {info['n_channels']} channels, {wl.n_cells} cells, T={wl.n_steps}, "
        f"workspace {info['workspace_bytes'] / 2**20:.1f} MiB")

    for w in range(args.warmup):
        r = prob.solve(workspace=ws, **opts)
        log(f"[bench] warmup {w}: force {r['force']:.10e} device {r['device_ms']:.1f} ms")

    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        t1 = time.perf_counter()
        r = prob.solve(workspace=ws, **opts)
        lat.append((time.perf_counter() - t1) * 1e3)
        log(f"[bench] step {k}: {lat[-1]:.1f} ms force {r['force']:.10e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cu_per_solve = r["cell_updates"]
    value = cu_per_solve * args.steps / elapsed

    # dominant kernel: field update, timed live with HIP events on the solve's stream
    rt = prob.solve(workspace=ws, time_stencil=True, **opts)
    avg_s = rt["stencil_ms_avg"] * 1e-3
    achieved = rt["stencil_alg_bytes"] / avg_s / 1e9 if avg_s > 0 else None
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": None,
                "kernel": "k_rb2d: fused register-blocked 2D update of all TM (or TE) channels, "
                          "steps_per_launch time steps per launch",
                "avg_launch_ms": rt["stencil_ms_avg"], "launches_timed": rt["stencil_samples"],
                "alg_bytes_per_launch": rt["stencil_alg_bytes"],
                "alg_bytes_per_cell_update": rt["stencil_alg_bytes"] / rt["stencil_cell_updates"],
                "tile_variant": rt["tile_variant"], "steps_per_launch": rt["tile_halo"]}

    out = {"metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"2D TE+TM piston force solve {wl.shape[0]}x{wl.shape[1]} res 40 "
                                  f"h=0.5, {info['n_channels']} channels, T={wl.n_steps}, sigma=1, "
                                  "courant 0.5, FP32 fields + FP64 surface/time accumulation",
                      "path": "batched", "channels": info["n_channels"], "cells": wl.n_cells,
                      "time_steps": wl.n_steps},
           "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                          "n": len(lat)},
           "force": r["force"], "roofline": roofline}

    # every fused-kernel variant on the same solve (T = 1000), the autotuner's
    # search space; all variants give bitwise-identical results
    sweep = []
    for v in range(1, 32):
        try:
            rv = prob.solve(workspace=ws, tile_variant=v, **dict(opts, n_steps=1000))
        except cf.CfError:
            break
        if not rv["fused"] or rv["tile_variant"] != v:
            break
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rv = prob.solve(workspace=ws, tile_variant=v, **dict(opts, n_steps=1000))
        sweep.append({"variant": v, "steps_per_launch": rv["tile_halo"],
                      "ms_per_1000_steps": (time.perf_counter() - t1) * 1e3})
    out["tile_sweep"] = sweep

    if not args.no_batch:
        # batching extension: the 24-clearance uneven piston set (h in [0.1, 2],
        # grid heights 84..160) in one batched launch sequence vs one problem
        # after another (each fused), T = 1000 steps
        from casimir_inputs import c3_uneven_set
        set_wl = [w.replace(n_steps=1000) for w in c3_uneven_set()]
        probs = [cf.Problem.from_workload(w) for w in set_wl]
        bo = dict(opts, n_steps=1000)
        cf.batch_solve(probs, **bo)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rb = cf.batch_solve(probs, **bo)
        tb = time.perf_counter() - t1
        cu = sum(r["cell_updates"] for r in rb)
        for p_ in probs:
            p_.solve(**bo)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for p_ in probs:
            p_.solve(**bo)
        ts = time.perf_counter() - t1
        out["batched_uneven"] = {"workload": "24 TE+TM pistons, h = linspace(0.1, 2.0), 400 x (84..160), "
                                             f"{sum(r['n_channels'] for r in rb)} channels, T=1000, FP32",
                                 "value": cu / tb, "unit": "cell-updates/s", "ms": tb * 1e3,
                                 "sequential_ms": ts * 1e3, "speedup_vs_sequential": ts / tb}

    gold = os.path.join(ROOT, "tests", "golden", "c2_piston_tetm_oracle.json")
    if os.path.exists(gold) and not args.n_steps:
        ref = json.load(open(gold))
        out["force_rel_err_vs_fp64_oracle"] = abs(r["force"] / ref["force"] - 1)

    if not args.no_plain:
        # plain path: one channel at a time, three launches per step; one TM
        # and one TE channel timed over the full T and scaled per cell-update
        n_tm = info["n_channels"] // 2          # TM channels come first
        sub = [0, n_tm]
        rp = prob.solve(workspace=ws, path="plain", channel_subset=sub, **opts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rp = prob.solve(workspace=ws, path="plain", channel_subset=sub, **opts)
        dtp = time.perf_counter() - t1
        plain_rate = rp["cell_updates"] / dtp
        out["plain"] = {"value": plain_rate, "unit": "cell-updates/s",
                        "sample": f"channels {sub} x {wl.n_steps} steps, plain path",
                        "projected_solve_ms": cu_per_solve / plain_rate * 1e3}
        out["speedup_vs_plain"] = value / plain_rate

    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
