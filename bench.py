"""Benchmark: Yee cell-updates/s of the batched FP32 force solve, force-solve
latency percentiles, and the plain one-channel-at-a-time path beside it.

One step = one complete force solve of the 2D TE+TM piston at 400 x 200
(res 40, h = 0.5, 40 cosine harmonics per face clamped to the face's sample
count -> 448 channels, T = 10000 time steps, sigma = 1, Courant 0.5): every
channel is kicked, advanced T steps and its surface correlation integrated
against K(t); the force is reduced on the host.  Inputs (material grids,
tables) are uploaded inside each solve; the timed work is the whole solve.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-plain]
                    [--no-batch] [--no-serve] [--serve-n N] [--serve-mixed]

Beside the headline line it measures the 3D path on the 192^3 sphere-plate
cell (a channel sample), the batched uneven piston set, and the serving
scheduler on a seeded stream of piston requests (saturated, then Poisson
arrivals at 0.7 of the measured capacity).

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


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_k_rb2d_piston2d_400x200_tetm_fp32.json")


def kernel_source_hash():
    """sha256 over the sources of the 2D kernels (the counters of a traffic
    record only hold for the code they were taken on)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels2d.hip", "device.hpp", "yee_common.hpp"):
        with open(os.path.join(ROOT, "paper_0906_5170_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(variant):
    """HBM bytes per launch of the fused kernel from the committed counter
    record (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter on a
    plain copy of known size), or None when the record does not match the
    current kernel source or variant."""
    if not os.path.exists(TRAFFIC_RECORD):
        return None, "no counter record"
    rec = json.load(open(TRAFFIC_RECORD))
    if rec.get("source_sha256") != kernel_source_hash():
        return None, "kernel source changed since the counters were taken"
    if rec.get("tile_variant") != variant:
        return None, f"counters taken on variant {rec.get('tile_variant')}, not {variant}"
    return rec["hbm_bytes_per_launch"], rec.get("command", "")


VALU_RECORD = os.path.join(ROOT, "profiles", "valu_k_rb2d_piston2d_400x200_tetm_fp32.json")
# VALU issue ceiling: 256 CUs x 4 SIMDs, each issuing one wave64 vector
# instruction every 4 cycles (16 lanes per SIMD), at 2.4 GHz
VALU_PEAK_WAVE_INSTR = 256 * 4 * 2.4e9 / 4
# lane-level VALU instructions of one 2D cell-update in the fused kernel's
# step arithmetic (TM and TE alike: the differences, the DPP neighbour moves,
# and a multiply and an FMA per updated component)
STEP_LANE_INSTR = 13


def measured_valu(variant):
    """Wave-level VALU instructions per launch of the fused 2D kernel
    (SQ_INSTS_VALU, mean over the TM and TE kernels) from the committed
    counter record, or None when it does not match the source or variant."""
    if not os.path.exists(VALU_RECORD):
        return None, "no counter record"
    rec = json.load(open(VALU_RECORD))
    if rec.get("source_sha256") != kernel_source_hash():
        return None, "kernel source changed since the counters were taken"
    if rec.get("tile_variant") != variant:
        return None, f"counters taken on variant {rec.get('tile_variant')}, not {variant}"
    return rec["valu_wave_instr_per_launch"], rec.get("command", "")


TRAFFIC_RECORD_3D = os.path.join(ROOT, "profiles", "traffic_k_f3d2_sphere_plate_192_fp32.json")


def kernel3d_source_hash():
    """sha256 over the sources of the fused 3D kernels."""
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels3d.hip", "device.hpp", "yee_common.hpp"):
        with open(os.path.join(ROOT, "paper_0906_5170_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic_3d(variant):
    """HBM bytes per launch of the fused 3D kernel from its committed counter
    record, or None when the record does not match the source or variant."""
    if not os.path.exists(TRAFFIC_RECORD_3D):
        return None, "no counter record"
    rec = json.load(open(TRAFFIC_RECORD_3D))
    if rec.get("source_sha256") != kernel3d_source_hash():
        return None, "kernel source changed since the counters were taken"
    if rec.get("tile_variant") != variant:
        return None, f"counters taken on variant {rec.get('tile_variant')}, not {variant}"
    return rec["hbm_bytes_per_launch"], rec.get("command", "")


SERVING_MIXED_RECORD = os.path.join(ROOT, "profiles", "serving_mixed_stream_first20.json")


def serving_source_hash():
    """sha256 over the scheduler and the kernels it launches."""
    import hashlib
    h = hashlib.sha256()
    for name in ("server.cpp", "kernels2d.hip", "kernels3d.hip", "device.hpp"):
        with open(os.path.join(ROOT, "paper_0906_5170_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_serving_mixed():
    """The committed record of the mixed 2D/3D stream served at its drawn
    sizes (bench.py --serve-mixed 20: about 13 minutes of GPU time, too long
    for the default run), with whether the scheduler and kernels are still
    the ones it was measured on."""
    if not os.path.exists(SERVING_MIXED_RECORD):
        return None
    rec = json.load(open(SERVING_MIXED_RECORD))
    rec["source_current"] = rec.get("source_sha256") == serving_source_hash()
    rec["measured_in_this_run"] = False
    return rec


C4_FULL_RECORD = os.path.join(ROOT, "profiles", "c4_full_solve_sphere_plate_192_fp32.json")


def measured_c4_full():
    """The committed record of the whole 3D force solve (bench.py --c4-full:
    about 4.5 minutes, too long for the default run), with whether the 3D
    kernel sources are still the ones it was measured on."""
    if not os.path.exists(C4_FULL_RECORD):
        return None
    rec = json.load(open(C4_FULL_RECORD))
    rec["source_current"] = rec.get("source_sha256") == kernel3d_source_hash()
    rec["measured_in_this_run"] = False
    return rec


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(wl, n_channels=32, n_steps=None):
    """The FP64 oracle as it stands, on a bounded sample of the workload:
    n_channels channels (spread over kinds, faces and polarizations) for
    n_steps steps, one process per channel on the host cores."""
    import oracle
    from oracle.force import setup
    _, _, _, _, chans = setup(wl)
    n_steps = n_steps or wl.n_steps
    pick = np.linspace(0, len(chans) - 1, n_channels).astype(int).tolist()
    workers = min(len(pick), os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    oracle.solve(wl, n_steps=n_steps, channel_subset=pick, workers=workers, chunk=1)
    dt = time.perf_counter() - t0
    cu = len(pick) * wl.n_cells * n_steps
    return {"value": cu / dt, "unit": "cell-updates/s", "cores": workers, "kind": "oracle",
            "host_cpu_count": os.cpu_count(), "per_core": cu / dt / workers,
            "sample": f"{len(pick)} of {len(chans)} channels x {n_steps} of {wl.n_steps} steps "
                      f"({cu:.3e} cell-updates, {dt:.1f} s, FP64 NumPy, one process per channel)"}


def cpu_baseline_reduced():
    """The oracle on bounded samples of the two reduced workloads of the
    benchmark (one process each), projected to a whole force point: the
    cylindrical piston (order 0, all channels, 300 steps) and the k_z
    dielectric piston (one k point, all channels, 200 steps)."""
    from casimir_inputs import c_cyl_piston, dielectric_piston2d, kz_gauss, kz_workload
    from oracle import cylforce, kz
    from oracle.cyl import cylindrical_courant
    from oracle.force import setup
    out = {}
    wl = c_cyl_piston()
    faces, bases, eps_s, mu_s, chans = cylforce.setup(wl)
    n_s = 300
    t1 = time.perf_counter()
    cylforce.run_order(wl, 0, faces, bases, eps_s, mu_s, chans, n_s, cylindrical_courant(wl.courant, 0))
    dt = time.perf_counter() - t1
    per = dt / (len(chans) * n_s)                  # seconds per channel-step
    total = sum(len(chans) * round(wl.n_steps * wl.courant / cylindrical_courant(wl.courant, m))
                for m in range(wl.m_max + 1))
    out["cylindrical"] = {"projected_force_point_s": per * total, "cores": 1,
                          "sample": f"order 0, all {len(chans)} channels x {n_s} steps, {dt:.1f} s, FP64 NumPy"}
    base = dielectric_piston2d(80, 40, 10, 20, 10, 20, 15, 20.0, n_steps=2000, n_harm=16, precision="fp32")
    ks, ws = kz_gauss(8, 12.0)
    wl = kz_workload(base, ks, ws)
    _, _, _, _, chans = setup(wl)
    n_s = 200
    t1 = time.perf_counter()
    kz.solve(wl.replace(n_steps=n_s), [ks[3]], [1.0])
    dt = time.perf_counter() - t1
    per = dt / (len(chans) * n_s)
    out["kz"] = {"projected_s": per * len(chans) * len(ks) * wl.n_steps, "cores": 1,
                 "sample": f"one k_z, all {len(chans)} channels x {n_s} steps, {dt:.1f} s, FP64 NumPy"}
    return out


def bench_3d(cf, torch, n_chan=64, n_steps=200, variant=0):
    """3D FP32 path on the 192^3 sphere-over-indented-plate cell (16-cell z
    CPML): a sample of n_chan of its 1280 channels, spread over faces, kinds
    and harmonics, for n_steps steps, all resident at once."""
    from casimir_inputs import c4_sphere_plate
    wl = c4_sphere_plate()
    p = cf.Problem.from_workload(wl)
    o = dict(sigma=wl.sigma, courant=wl.courant, n_steps=n_steps, pol=wl.pol, kernel=wl.kernel,
             precision="fp32", tile_variant=variant)
    C = p.info(**o)["n_channels"]
    sub = np.linspace(0, C - 1, n_chan).astype(int).tolist()
    p.solve(channel_subset=sub, **dict(o, n_steps=10))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r = p.solve(channel_subset=sub, time_stencil=True, **o)
    dt = time.perf_counter() - t1
    ceiling = HBM_PEAK_GBS * 1e9 / 48.0       # 48 B per 3D FP32 cell-update
    rate = r["cell_updates"] / dt
    sweep = []
    for v in (range(0, 7) if not variant else ()):   # 0: split half-step kernels, 1..6: fused variants
        ov = dict(o, n_steps=60)
        ov.update(split=True) if v == 0 else ov.update(tile_variant=v)
        rv = p.solve(channel_subset=sub, time_stencil=True, **ov)
        if v and (not rv["fused"] or rv["tile_variant"] != v):
            continue
        cu_s = rv["stencil_cell_updates"] / (rv["stencil_ms_avg"] * 1e-3) if rv["stencil_ms_avg"] else None
        sweep.append({"variant": v, "fused": rv["fused"], "stencil_cell_updates_per_s": cu_s})
    step_rate = r["stencil_cell_updates"] / (r["stencil_ms_avg"] * 1e-3) if r["stencil_ms_avg"] else None
    traffic, traffic_note = measured_traffic_3d(r["tile_variant"])
    # cells the fused steps advance per launch (planes below the conductor skipped)
    adv = r["stencil_cell_updates"] * r["advanced_cell_updates"] / r["cell_updates"]
    log(f"[bench] 3d: {rate:.3e} cell-updates/s over the solve, stencil {step_rate:.3e}, "
        f"advanced {adv / r['stencil_cell_updates']:.3f} of the cells")
    return {"workload": f"sphere over indented plate 192^3 res 48, z CPML 16, {n_chan} of {C} channels "
                        f"x {n_steps} steps, FP32 fields", "value": rate, "unit": "cell-updates/s",
            "stencil_cell_updates_per_s": step_rate,
            "stencil_frac_of_hbm_ceiling": step_rate / ceiling if step_rate else None,
            "hbm_ceiling_cell_updates_per_s": ceiling, "fused": r["fused"], "variant": r["tile_variant"],
            "avg_launch_ms": r["stencil_ms_avg"], "cell_updates_per_launch": r["stencil_cell_updates"],
            "advanced_cell_updates_per_launch": adv,
            "advanced_cell_updates_per_s": r["advanced_cell_updates"] / dt,
            "traffic_bytes_per_launch": traffic, "traffic_note": traffic_note,
            "traffic_bytes_per_advanced_cell_update": traffic / adv if traffic else None,
            "real_hbm_GBps": traffic / (r["stencil_ms_avg"] * 1e-3) / 1e9 if traffic and r["stencil_ms_avg"] else None,
            "variant_sweep": sweep,
            "projected_full_solve_s": 1280 * wl.n_cells * wl.n_steps / rate,
            "full_solve_record": measured_c4_full()}


def bench_3d_full(cf, torch, waves=3, precision="fp32", run=None):
    """The whole 3D sphere-over-indented-plate force solve (192^3, 1280
    channels, T = 6000, FP32 fields): the channels in `waves` equal channel
    waves, each all resident on the GPU (about 160 GB each), one solve per
    wave; the force is the sum of the waves' forces (it is linear in the
    channels)."""
    from casimir_inputs import c4_sphere_plate
    wl = c4_sphere_plate()
    p = cf.Problem.from_workload(wl)
    o = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol=wl.pol, kernel=wl.kernel,
             precision=precision)
    C = p.info(**o)["n_channels"]
    parts = np.array_split(np.arange(C), waves)
    ws = torch.empty(p.info(**dict(o, max_resident=len(parts[0])))["workspace_bytes"], dtype=torch.uint8,
                     device="cuda")
    force, cu, adv, dev_ms = 0.0, 0.0, 0.0, 0.0
    t0 = time.perf_counter()
    run = list(range(waves)) if run is None else list(run)
    for k, sub in enumerate(parts):
        if k not in run:
            continue
        r = p.solve(workspace=ws, channel_subset=sub.tolist(), max_resident=len(sub), **o)
        force += r["force"]
        cu += r["cell_updates"]
        adv += r["advanced_cell_updates"]
        dev_ms += r["device_ms"]
        log(f"[bench] c4 full: wave {k + 1}/{waves} ({len(sub)} channels) {r['device_ms'] / 1e3:.1f} s, "
            f"variant {r['tile_variant']}, partial force {r['force']:+.6e}")
    wall = time.perf_counter() - t0
    return {"workload": f"sphere over indented plate 192^3 res 48, z CPML 16, all {C} channels x {wl.n_steps} "
                        f"steps, {precision.upper()} fields, {waves} channel waves", "waves_run": run,
            "force": force, "wall_s": wall,
            "device_s": dev_ms / 1e3, "cell_updates": cu, "value": cu / (dev_ms * 1e-3),
            "advanced_cell_updates": adv, "advanced_cell_updates_per_s": adv / (dev_ms * 1e-3),
            "unit": "cell-updates/s", "workspace_bytes": ws.numel()}


def bench_cyl(cf, torch, quick=False):
    """Cylindrical piston (Sec. III C, Fig. 7) at resolution 40, n, m in
    {0, 1, 2}: one whole force point (126 channels; orders 0 and 1 take
    10000 steps, order 2 15000 on its smaller step) at the default FP64
    fields on the resident kernel; the split half-step path and FP32 fields
    (a stated-error option: its channel terms cancel by 3e8, see the
    precision record) beside it.  The paper quotes about 5 minutes on 8
    processors per such force point (2009 CPUs, time span unstated)."""
    from casimir_inputs import c_cyl_piston
    wl = c_cyl_piston()
    p = cf.Problem.from_workload(wl)
    o = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol="3D", kernel=wl.kernel,
             precision=wl.precision)
    p.solve(**dict(o, n_steps=200))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r = p.solve(time_stencil=True, **o)
    wall = time.perf_counter() - t1
    rate = r["cell_updates"] / (r["device_ms"] * 1e-3)
    if quick:
        return {"force": r["force"], "device_ms": r["device_ms"], "value": rate, "unit": "cell-updates/s",
                "resident_variant": r["tile_variant"], "launch_ms": r["stencil_ms_avg"]}
    rs = p.solve(split=True, **o)
    r32 = p.solve(**dict(o, precision="fp32"))
    fsz = 8.0 if wl.precision == "fp64" else 4.0
    alg = rate * 12.0 * fsz                            # read + write of 6 field values per cell-update
    out = {"workload": f"cylindrical piston res 40, h 0.5, tube {wl.shape[0]} x {wl.shape[1]} (z x r), "
                       f"n_harm 3, m 0..2, {r['n_channels']} channels, T 10000 (order 2: 15000), "
                       f"{wl.precision.upper()} fields",
           "precision": wl.precision, "force": r["force"], "force_fp32_fields": r32["force"],
           "force_point_wall_s": wall, "device_ms": r["device_ms"], "value": rate, "unit": "cell-updates/s",
           "resident_variant": r["tile_variant"], "split_path_device_ms": rs["device_ms"],
           "speedup_vs_split": rs["device_ms"] / r["device_ms"], "fp32_device_ms": r32["device_ms"],
           "fp32_resident_variant": r32["tile_variant"],
           "alg_bytes_per_s": alg, "alg_frac_of_hbm_peak": alg / (HBM_PEAK_GBS * 1e9),
           "paper_quote": "about 5 minutes per force point on 8 processors (2009), res 40, n,m in {0,1,2}"}
    log(f"[bench] cyl: force point {wall:.3f} s wall ({r['device_ms']:.1f} ms device, {wl.precision}), "
        f"{rate:.3e} cell-updates/s, split {rs['device_ms']:.1f} ms, fp32 {r32['device_ms']:.1f} ms")
    # a sweep of four clearances: one at a time, then as one batch (the
    # reduced solves run concurrently and share the CUs a single force point
    # leaves idle)
    hs = [0.4, 0.5, 0.6, 0.7]
    sweep = [cf.Problem.from_workload(c_cyl_piston(h_u=h)) for h in hs]
    cf.batch_solve(sweep, **dict(o, n_steps=200))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    seq = [q.solve(**o)["force"] for q in sweep]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t1
    t1 = time.perf_counter()
    bat = [x["force"] for x in cf.batch_solve(sweep, **o)]
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t1
    assert bat == seq, (bat, seq)
    out["sweep4"] = {"clearances": hs, "one_at_a_time_wall_s": t_seq, "batched_wall_s": t_bat,
                     "force_points_per_s": len(hs) / t_bat, "speedup": t_seq / t_bat}
    log(f"[bench] cyl sweep of {len(hs)} clearances: {t_seq:.3f} s one at a time, {t_bat:.3f} s batched "
        f"({len(hs) / t_bat:.1f} force points/s)")
    return out


def bench_kz(cf, torch):
    """z-invariant dielectric piston (eps = 4 blocks between PEC slabs; the
    C1 geometry: res 20, 80 x 40, 16 harmonics, T = 2000) integrated over
    k_z with 8-point Gauss-Legendre on [0, 12] (Sec. III B: dielectrics
    hybridize the polarizations): 8 six-component runs in one launch, FP32."""
    from casimir_inputs import dielectric_piston2d, kz_gauss, kz_workload
    base = dielectric_piston2d(80, 40, 10, 20, 10, 20, 15, 20.0, n_steps=2000, n_harm=16, precision="fp32")
    ks, ws = kz_gauss(8, 12.0)
    wl = kz_workload(base, ks, ws)
    p = cf.Problem.from_workload(wl)
    o = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol="3D", kernel="general", precision="fp32")
    p.solve(**dict(o, n_steps=100))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r = p.solve(time_stencil=True, **o)
    wall = time.perf_counter() - t1
    rate = r["cell_updates"] / (r["device_ms"] * 1e-3)
    rs = p.solve(split=True, **o)
    out = {"workload": f"dielectric piston (eps 4) res 20, 80 x 40, 16 harmonics, k_z 8-point Gauss on [0, 12], "
                       f"{r['n_channels']} channels, T 2000, FP32",
           "force_per_length": r["force"], "wall_s": wall, "device_ms": r["device_ms"], "value": rate,
           "unit": "cell-updates/s", "resident_variant": r["tile_variant"],
           "split_path_device_ms": rs["device_ms"], "speedup_vs_split": rs["device_ms"] / r["device_ms"],
           "alg_bytes_per_s": rate * 48.0, "alg_frac_of_hbm_peak": rate * 48.0 / (HBM_PEAK_GBS * 1e9)}
    # Bloch-periodic x (complex fields): dielectric blocks repeated with period
    # 2.4 above a PEC plate, 8 k_x points on [0, pi/L) x 4 k_z points
    from casimir_inputs.geometry import Box, Workload, rasterize
    big = 1e30
    nx, ny = 48, 60
    prims = [Box((-big, -big, -big), (big, 8, big), 1), Box((16, 24, -big), (32, 36, big), 2)]
    gw = Workload(name="grating", ndim=2, shape=(nx, ny, 1), res=20.0, bc=("periodic", "pec", "periodic"),
                  pml_cells=(0, 0, 0), eps=[1.0, float("-inf"), 4.0], mu=[1.0, 1.0, 1.0],
                  comp_ids=rasterize((nx, ny, 1), prims), s_lo=(12, 20, 0), s_hi=(36, 40, 1), n_harm=8,
                  force_axis=1, pol="3D", kernel="general", n_steps=2000, sigma=1.0, courant=0.5, precision="fp32")
    Lx = nx / gw.res
    kxs = (np.arange(8) + 0.5) * (np.pi / Lx) / 8
    kzs, kzw = kz_gauss(4, 12.0)
    pts = [(kx, kz) for kx in kxs for kz in kzs]
    wts = [w / len(kxs) for _ in kxs for w in kzw]     # zone average over k_x (F(-k_x) = F(k_x)), k_z integral
    bw = kz_workload(gw, [p[1] for p in pts], wts, kx=[p[0] for p in pts])
    pb = cf.Problem.from_workload(bw)
    ob = dict(sigma=1.0, courant=0.5, n_steps=2000, pol="3D", kernel="general", precision="fp32")
    pb.solve(**dict(ob, n_steps=50))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rb = pb.solve(**ob)
    wb = time.perf_counter() - t1
    rate_b = rb["cell_updates"] / (rb["device_ms"] * 1e-3)
    out["bloch"] = {"workload": f"grating: eps 4 blocks with period 2.4 above a PEC plate, res 20, 48 x 60 cell, "
                                f"8 k_x x 4 k_z points, {rb['n_channels']} complex channels, T 2000, FP32",
                    "force_per_length_per_cell": rb["force"], "wall_s": wb, "device_ms": rb["device_ms"], "value": rate_b,
                    "unit": "cell-updates/s (complex cells)", "resident_variant": rb["tile_variant"],
                    "alg_bytes_per_s": rate_b * 96.0, "alg_frac_of_hbm_peak": rate_b * 96.0 / (HBM_PEAK_GBS * 1e9)}
    log(f"[bench] bloch: {wb:.3f} s wall ({rb['device_ms']:.1f} ms device), {rate_b:.3e} complex cell-updates/s")
    log(f"[bench] kz: {wall:.3f} s wall ({r['device_ms']:.1f} ms device), {rate:.3e} cell-updates/s, "
        f"split {rs['device_ms']:.1f} ms")
    out["open_space"] = bench_open_space(cf, torch)
    return out


def bench_open_space(cf, torch):
    """Sec. III B's dispersive computation: two silicon-like waveguides (eps_inf
    1.035 plus one Lorentz term of strength 10.835 at w0 = 22, a length unit
    of 1 um) of 0.5 x 0.25 cross-section, 0.25 apart, in vacuum closed by a
    0.5-thick CPML on all four sides; res 40 (130 x 90 cells), 8 harmonics
    per face, k_z by 8-point Gauss-Legendre on [0, 16], T = 8000.  Split
    kernels (in-plane CPML and polarizations); FP32 fields timed, the FP64
    fields force beside it."""
    from casimir_inputs import kz_gauss, kz_workload, waveguides_open_2d
    base = waveguides_open_2d(40, 0.5, 0.25, 0.25, 0.5, 0.5, 1.035, ((10.835, 22.0),), n_harm=8,
                              n_steps=8000, precision="fp32")
    ks, ws = kz_gauss(8, 16.0)
    wl = kz_workload(base, ks, ws)
    p = cf.Problem.from_workload(wl)
    o = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol="3D", kernel="general", precision="fp32")
    p.solve(**dict(o, n_steps=50))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r = p.solve(**o)
    wall = time.perf_counter() - t1
    r64 = p.solve(**dict(o, precision="fp64"))
    rate = r["cell_updates"] / (r["device_ms"] * 1e-3)
    rec = {"workload": f"two silicon-like waveguides 0.5 x 0.25, gap 0.25, in vacuum with CPML on four sides, res 40, "
                       f"{wl.shape[0]} x {wl.shape[1]}, 8 harmonics per face, k_z 8-point Gauss on [0, 16], "
                       f"{r['n_channels']} channels, T {wl.n_steps}, FP32 fields",
           "force_per_length": r["force"], "force_per_length_fp64_fields": r64["force"],
           "fp32_vs_fp64_fields_rel": abs(r["force"] / r64["force"] - 1),
           "wall_s": wall, "device_ms": r["device_ms"], "device_ms_fp64": r64["device_ms"], "value": rate,
           "unit": "cell-updates/s", "path": "split half-step kernels (CPML and Lorentz polarizations)",
           "alg_bytes_per_s": rate * 48.0, "alg_frac_of_hbm_peak": rate * 48.0 / (HBM_PEAK_GBS * 1e9)}
    log(f"[bench] open space (Sec. III B waveguides): {wall:.2f} s wall ({r['device_ms']:.0f} ms device), "
        f"{rate:.3e} cell-updates/s, force {r['force']:.6e} (FP64 fields {r64['force']:.6e})")
    return rec


def _serve(cf, srv_budget, reqs, probs, opts_list, lam_times=True, keep=None):
    """Submit requests at their arrival times (or all at once) and collect
    them as they finish; returns per-request rows (kind, submit, admit,
    done, cell-updates) in stream order, and the results of the requests
    whose stream indices are in keep.  Latencies come from the server's own
    clock (cf_server_times), so the polling interval does not enter them."""
    rows = [None] * len(reqs)
    kept = {}
    with cf.Server(srv_budget) as srv:
        t0 = time.perf_counter()
        pending = {}
        nxt = 0
        last = t0
        while nxt < len(reqs) or pending:
            now = time.perf_counter() - t0
            while nxt < len(reqs) and (not lam_times or reqs[nxt].t_arrive <= now):
                q, p, o = reqs[nxt], probs[nxt], opts_list[nxt]
                try:
                    pending[srv.submit(p, **o)] = nxt
                except cf.CfError as e:
                    rows[nxt] = dict(kind=q.kind, rejected=True, index=q.index)
                    log(f"[bench] serve: request {q.index} rejected: {e}")
                nxt += 1
            for t in list(pending):
                state, r = srv.poll(t)
                if state in ("failed", "cancelled"):
                    raise RuntimeError(f"served request {reqs[pending[t]].index} {state}")
                if state != "done":
                    continue
                k = pending.pop(t)
                q = reqs[k]
                ts, ta, td = srv.times(t)
                rows[k] = dict(kind=q.kind, index=q.index, submit=ts, admit=ta, done=td, cu=r["cell_updates"],
                               fused=r["fused"], rejected=False, steps=r["n_steps_run"],
                               t_full=opts_list[k]["n_steps"])
                if keep is not None and q.index in keep:
                    kept[q.index] = r
                srv.release(t)
                last = time.perf_counter()
                if len(reqs) <= 40 or q.kind != "2d":
                    log(f"[bench] serve: request {q.index} ({q.kind}) done, latency {td - ts:.2f} s")
            if time.perf_counter() - last > 60:
                st = srv.stats()
                log(f"[bench] serve: {st['completed']} done, {st['running']} resident, {st['queued']} queued, "
                    f"scheduler clock {st['clock_steps']} steps")
                last = time.perf_counter()
            wait = 0.2
            if lam_times and nxt < len(reqs):
                wait = min(wait, max(reqs[nxt].t_arrive - (time.perf_counter() - t0), 0.0))
            time.sleep(wait)
    return (rows, kept) if keep is not None else rows


def _summary(rows):
    ok = [r for r in rows if not r["rejected"]]
    lat = np.array([r["done"] - r["submit"] for r in ok])
    wait = np.array([r["admit"] - r["submit"] for r in ok])
    span = max(r["done"] for r in ok) - min(r["submit"] for r in ok)
    out = {"n": len(ok), "rejected": len(rows) - len(ok),
           "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
           "mean_queue_wait_s": float(wait.mean()), "span_s": span,
           "cell_updates_per_s": sum(r["cu"] for r in ok) / span,
           "fused_requests": sum(1 for r in ok if r["fused"]),
           "steps_run_fraction": sum(r["steps"] for r in ok) / sum(r["t_full"] for r in ok)}
    for kind in sorted({r["kind"] for r in rows}):
        lk = np.array([r["done"] - r["submit"] for r in ok if r["kind"] == kind])
        if len(lk):
            out[f"{kind}_p50_s"] = float(np.percentile(lk, 50))
            out[f"{kind}_p99_s"] = float(np.percentile(lk, 99))
        if len({r["kind"] for r in rows}) > 1:
            out[f"{kind}_n"] = len(lk)
            out[f"{kind}_rejected"] = sum(1 for r in rows if r["rejected"] and r["kind"] == kind)
            out[f"{kind}_cell_updates"] = float(sum(r["cu"] for r in ok if r["kind"] == kind))
    return out


def bench_serving(cf, torch, args, rate_3d):
    """Serving on the seeded piston class of the mixed request stream: every
    request is a complete force solve (2D TE+TM piston, clearance
    h ~ U[0.1, 2], resolution ~ U{20..60}, T = 250 res, FP32).  First all
    requests at once (saturation: the server's capacity), then the same
    requests arriving as a Poisson stream at 0.7 of that capacity (the
    load-matched stream whose latency percentiles are the headline)."""
    from casimir_inputs.streams import mixed_stream, rescale_arrivals
    budget = int(min(torch.cuda.get_device_properties(0).total_memory * 0.6, 160 * 2**30))
    reqs, wls, probs = [], [], []
    for q in mixed_stream(2 * args.serve_n, lam=4.0, seed=0, kinds=["2d"]):
        w = q.workload()
        try:
            p_ = cf.Problem.from_workload(w)
        except cf.CfError:          # no room for S between block and sidewall
            continue
        reqs.append(q)
        wls.append(w)
        probs.append(p_)
        if len(reqs) == args.serve_n:
            break
    opts = [dict(sigma=w.sigma, courant=w.courant, n_steps=w.n_steps, pol=w.pol, kernel=w.kernel,
                 precision="fp32") for w in wls]
    log(f"[bench] serve: {len(reqs)} piston requests, saturated pass ...")
    sat = _summary(_serve(cf, budget, reqs, probs, opts, lam_times=False))
    cap = sat["n"] / sat["span_s"]                       # requests per second at saturation
    lam = 0.7 * cap
    log(f"[bench] serve: capacity {cap:.2f} req/s; Poisson pass at {lam:.2f} req/s ...")
    matched = _summary(_serve(cf, budget, rescale_arrivals(reqs, lam), probs, opts))
    # the same requests with the time-convergence stop (FP32 noise floor 1e-6,
    # checked every 100 steps): all at once, then at 0.7 of that capacity
    stop_opts = [dict(o, stop_tol=1e-6, stop_every=100) for o in opts]
    sat_stop = _summary(_serve(cf, budget, reqs, probs, stop_opts, lam_times=False))
    cap_stop = sat_stop["n"] / sat_stop["span_s"]
    matched_stop = _summary(_serve(cf, budget, rescale_arrivals(reqs, 0.7 * cap_stop), probs, stop_opts))
    log(f"[bench] serve with stop: capacity {cap_stop:.2f} req/s, steps run {sat_stop['steps_run_fraction']:.2f}, "
        f"p50 {matched_stop['p50_s']:.3f} s p99 {matched_stop['p99_s']:.3f} s")
    res = {"stream": f"piston class of the seeded mixed stream (seed 0), {len(reqs)} requests: "
                     "clearance h ~ U[0.1,2], res ~ U{20..60}, T = 250 res, 40 harmonics/face, TE+TM, FP32",
           "budget_bytes": budget, "saturated": sat, "capacity_req_per_s": cap,
           "load_matched": dict(matched, lam_req_per_s=lam, load=0.7),
           "with_convergence_stop": {"stop_tol": 1e-6, "stop_every": 100, "saturated": sat_stop,
                                     "capacity_req_per_s": cap_stop,
                                     "load_matched": dict(matched_stop, lam_req_per_s=0.7 * cap_stop, load=0.7)}}
    # the literal mixed stream (4 req/s, 70 % pistons / 30 % 3D cells): offered
    # load against capacity from the measured per-class rates
    if rate_3d:
        lit = mixed_stream(200, lam=4.0, seed=0)
        rate_2d = sat["cell_updates_per_s"]
        svc, infeasible = [], 0
        for q in lit:
            if q.kind == "2d":
                w = q.workload()
                try:
                    c = cf.Problem.from_workload(w).info(**opts[0])["n_channels"]
                except cf.CfError:
                    infeasible += 1
                    continue
                svc.append(c * w.n_cells * w.n_steps / rate_2d)
            else:
                n = q.params["n"]
                svc.append(1280 * n ** 3 * (125 * n // 4) / rate_3d)
        res["literal_stream"] = {"lam_req_per_s": 4.0, "n": len(lit), "infeasible_2d": infeasible,
                                 "mean_service_s_estimated": float(np.mean(svc)),
                                 "offered_load_x_capacity": 4.0 * float(np.mean(svc)),
                                 "note": "service times from the measured saturated piston rate and the "
                                         "3D sample rate; the stream is far beyond one GPU's capacity, "
                                         "so its backlog grows without bound"}
    log(f"[bench] serve: p50 {matched['p50_s']:.3f} s p99 {matched['p99_s']:.3f} s")
    mixed = measured_serving_mixed()
    if mixed is not None:
        res["mixed"] = mixed
    return res


def bench_serving_mixed(cf, torch, args):
    """The first args.serve_mixed requests of the seeded mixed stream (seed
    0), both classes at their drawn sizes: 2D TE+TM pistons (FP32, T = 250
    res) and 3D sphere-above-indented-plate cells (n^3, n in {96, 128, 160,
    192}, T = 125 n / 4, 1280 channels).  3D requests whose gap leaves no room
    for the stress surface inside the indentation are rejected by the
    server (CF_E_SURFACE) and counted.  Passes: 'sat' submits everything at
    once (capacity = requests / span), 'check' solves the smallest served 3D
    request once more as a one-shot cf_solve with the served kernel variant
    and compares the per-channel integrals bit for bit, 'matched' replays the
    requests as a Poisson stream at 0.7 of the capacity (or at
    --serve-mixed-lam requests per second)."""
    from casimir_inputs.streams import mixed_stream, rescale_arrivals
    passes = args.serve_mixed_passes.split(",")
    budget = int(min(torch.cuda.get_device_properties(0).total_memory * 0.8, 224 * 2**30))
    reqs, probs, opts, built_rejects = [], [], [], []
    for q in mixed_stream(args.serve_mixed, lam=4.0, seed=0):
        w = q.workload()
        try:
            p_ = cf.Problem.from_workload(w)
        except cf.CfError as e:
            built_rejects.append({"index": q.index, "kind": q.kind, "error": str(e)})
            continue
        reqs.append(q)
        probs.append(p_)
        opts.append(dict(sigma=w.sigma, courant=w.courant, n_steps=w.n_steps, pol=w.pol,
                         kernel=w.kernel, precision="fp32"))
    n3 = sum(1 for q in reqs if q.kind == "3d")
    log(f"[bench] serve mixed: {len(reqs)} requests ({n3} 3D), budget {budget / 2**30:.0f} GiB")
    res = {"stream": f"first {args.serve_mixed} requests of the seeded mixed stream (seed 0): 2D TE+TM pistons "
                     "(h ~ U[0.1,2], res ~ U{20..60}, T = 250 res, 40 harmonics/face) and 3D sphere-above-"
                     "indented-plate cells (n^3, n ~ U{96,128,160,192}, gap ~ U[0.2,1.5], T = 125 n/4, "
                     "8x8 harmonics/face, 1280 channels), FP32 fields",
           "requests": [{"index": q.index, "kind": q.kind, **q.params} for q in reqs],
           "rejected_at_build": built_rejects, "budget_bytes": budget,
           "source_sha256": serving_source_hash()}
    cap = None
    if "sat" in passes or "check" in passes:
        log("[bench] serve mixed: saturated pass ...")
        rows, kept = _serve(cf, budget, reqs, probs, opts, lam_times=False,
                            keep={q.index for q in reqs if q.kind == "3d"})
        rej = [dict(kind=r["kind"], rejected=True) for r in built_rejects]
        sat = _summary(rows + rej)
        cap = sat["n"] / sat["span_s"]
        res["saturated"] = sat
        res["capacity_req_per_s"] = cap
        log(f"[bench] serve mixed: capacity {cap:.4f} req/s, {sat['cell_updates_per_s']:.3e} cell-updates/s, "
            f"3D p50 {sat.get('3d_p50_s', float('nan')):.1f} s, 2D p50 {sat.get('2d_p50_s', float('nan')):.2f} s")
        served3 = [q for q in reqs if q.index in kept]
        if "check" in passes and served3:
            small = min(served3, key=lambda q: q.params["n"])
            k = next(i for i, q in enumerate(reqs) if q.index == small.index)
            served = kept[small.index]
            one = probs[k].solve(**dict(opts[k], tile_variant=served["tile_variant"]))
            same = bool(np.array_equal(served["per_channel"], one["per_channel"])
                        and served["force"] == one["force"])
            res["bitwise_check"] = {"request": small.index, "n": small.params["n"],
                                    "tile_variant": served["tile_variant"], "fused": served["fused"],
                                    "force": served["force"], "one_shot_force": one["force"],
                                    "bitwise_equal": same}
            log(f"[bench] serve mixed: request {small.index} served == one-shot bit for bit: {same}")
            if not same:
                raise RuntimeError("served 3D request differs from its one-shot solve")
    if "matched" in passes:
        lam = args.serve_mixed_lam or (0.7 * cap if cap else None)
        if not lam:
            raise SystemExit("the matched pass needs the saturated pass or --serve-mixed-lam")
        log(f"[bench] serve mixed: Poisson pass at {lam:.4f} req/s ...")
        rej = [dict(kind=r["kind"], rejected=True) for r in built_rejects]
        m = _summary(_serve(cf, budget, rescale_arrivals(reqs, lam), probs, opts) + rej)
        res["load_matched"] = dict(m, lam_req_per_s=lam,
                                   load=(lam / cap) if cap else None)
        log(f"[bench] serve mixed: matched p50 {m['p50_s']:.1f} s p99 {m['p99_s']:.1f} s")
    return res


def bench_precision(cf, torch):
    """FP32 fields with FP64 accumulation against the stored FP64 oracle
    results (tests/golden), per configuration: relative force error (C1,
    C3 members) or relative channel-integral error (C4 sample channels over
    the full T).  The C2 headline error is reported beside the main line."""
    from casimir_inputs import c1_piston_tm_fp64, c3_uneven_set, c4_sphere_plate
    gdir = os.path.join(ROOT, "tests", "golden")
    res = {}

    def opts(wl, **over):
        o = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol=wl.pol, kernel=wl.kernel,
                 precision="fp32")
        o.update(over)
        return o
    path = os.path.join(gdir, "c1_piston_tm_oracle.json")
    if os.path.exists(path):
        ref = json.load(open(path))
        wl = c1_piston_tm_fp64()
        p = cf.Problem.from_workload(wl)
        r32 = p.solve(**opts(wl))
        r64 = p.solve(**opts(wl, precision="fp64"))
        res["c1"] = {"workload": "2D TM piston 80x40 res 20, T=2000",
                     "fp32_force_rel_err": abs(r32["force"] / ref["force"] - 1),
                     "fp64_force_rel_err": abs(r64["force"] / ref["force"] - 1)}
    path = os.path.join(gdir, "c3_uneven_members_oracle.json")
    if os.path.exists(path):
        ref = json.load(open(path))
        wls = c3_uneven_set()
        errs = []
        for m in ref["members"]:
            wl = wls[m["index"]]
            r = cf.Problem.from_workload(wl).solve(**opts(wl))
            errs.append({"member": m["index"], "h": m["h"], "shape": m["shape"],
                         "fp32_force_rel_err": abs(r["force"] / m["force"] - 1)})
        res["c3"] = {"workload": "uneven piston set members, 400 x (84 | 160), T=10000", "members": errs}
    path = os.path.join(gdir, "c4_sphere_plate_channels_full_T_oracle.json")
    if os.path.exists(path):
        ref = json.load(open(path))
        wl = c4_sphere_plate()
        r = cf.Problem.from_workload(wl).solve(channel_subset=ref["subset"], **opts(wl))
        acc_ref = np.array(ref["per_channel"])
        err = np.abs(r["per_channel"] - acc_ref) / np.abs(acc_ref)
        res["c4"] = {"workload": f"192^3 sphere-plate, channels {ref['subset']}, T={ref['n_steps']}",
                     "fp32_channel_rel_err_max": float(err.max()),
                     "fp32_channel_rel_err": [float(e) for e in err]}
    path = os.path.join(gdir, "cyl_piston_res40_oracle.json")
    if os.path.exists(path):
        from casimir_inputs import c_cyl_piston
        ref = json.load(open(path))
        wl = c_cyl_piston()
        p = cf.Problem.from_workload(wl)
        o = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol="3D", kernel=wl.kernel)
        r32 = p.solve(precision="fp32", **o)
        r64 = p.solve(precision="fp64", **o)
        acc_ref = np.array(ref["per_channel"])
        res["cylindrical"] = {"workload": "cylindrical piston res 40, n, m in {0, 1, 2}, T=10000",
                              "default_precision": wl.precision,
                              "default_force_rel_err": abs((r64 if wl.precision == "fp64" else r32)["force"]
                                                           / ref["force"] - 1),
                              "fp32_force_rel_err": abs(r32["force"] / ref["force"] - 1),
                              "fp64_force_rel_err": abs(r64["force"] / ref["force"] - 1),
                              "fp32_channel_err_of_largest": float(np.max(np.abs(r32["per_channel"] - acc_ref))
                                                                   / np.max(np.abs(acc_ref)))}
    path = os.path.join(gdir, "kz_dielectric_piston_oracle.json")
    if os.path.exists(path):
        from casimir_inputs import dielectric_piston2d, kz_workload
        ref = json.load(open(path))
        base = dielectric_piston2d(80, 40, 10, 20, 10, 20, 15, 20.0, n_steps=2000, n_harm=16)
        wl = kz_workload(base, ref["kz"], ref["kz_weight"])
        p = cf.Problem.from_workload(wl)
        o = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol="3D", kernel="general")
        r32 = p.solve(precision="fp32", **o)
        r64 = p.solve(precision="fp64", **o)
        res["kz"] = {"workload": "k_z dielectric piston 80x40 res 20, 8 k points, T=2000",
                     "fp32_force_rel_err": abs(r32["force"] / ref["force"] - 1),
                     "fp64_force_rel_err": abs(r64["force"] / ref["force"] - 1)}
    log(f"[bench] precision: {json.dumps(res)}")
    return res

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--stencil-only", action="store_true",
                    help="only the sampled-timing solve of the headline workload (its launches run one at a "
                         "time on one stream): the command for kernel traces of the dominant kernel")
    ap.add_argument("--main-only", action="store_true",
                    help="only the headline solve and its stencil timing (for counter runs)")
    ap.add_argument("--tile-variant", type=int, default=0,
                    help="fused kernel variant for the headline solve (0: autotuned)")
    ap.add_argument("--with-3d", action="store_true", help="run the 3D sample even with --main-only")
    ap.add_argument("--c4-steps", type=int, default=200, help="time steps of the 3D sample")
    ap.add_argument("--c4-full", action="store_true",
                    help="only the whole 3D sphere-plate force solve (1280 channels x 6000 steps, several "
                         "minutes), in channel waves that fit the GPU's memory")
    ap.add_argument("--c4-full-precision", default="fp32", choices=("fp32", "fp64"),
                    help="field precision of --c4-full")
    ap.add_argument("--c4-full-waves", type=int, default=0,
                    help="channel waves of --c4-full (0: 3 in FP32, 16 in FP64)")
    ap.add_argument("--c4-full-from", type=int, default=0, help="first wave of --c4-full to run")
    ap.add_argument("--c4-full-count", type=int, default=0,
                    help="waves of --c4-full to run (0: all from --c4-full-from on); the partial force of "
                         "the waves run is reported")
    ap.add_argument("--c4-variant", type=int, default=0,
                    help="fused 3D variant of the 3D sample (0: autotuned, with a sweep of all variants)")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-cyl", action="store_true")
    ap.add_argument("--cyl-only", action="store_true",
                    help="only the cylindrical piston section (for profiling); prints its record")
    ap.add_argument("--cyl-quick", action="store_true",
                    help="with --cyl-only: the register-resident FP32 solve only (no split / FP64 / oracle)")
    ap.add_argument("--open-only", action="store_true",
                    help="only the open-space waveguide pair (for profiling); prints its record")
    ap.add_argument("--serve-n", type=int, default=24, help="requests in the served piston stream")
    ap.add_argument("--serve-mixed", type=int, default=0,
                    help="only serve this many requests of the mixed 2D/3D stream at their drawn sizes "
                         "(long: 3D requests take up to minutes each) and print the record")
    ap.add_argument("--serve-mixed-passes", default="sat,check,matched",
                    help="passes of --serve-mixed: sat, check, matched")
    ap.add_argument("--serve-mixed-lam", type=float, default=0.0,
                    help="arrival rate of the matched pass (0: 0.7 of the saturated capacity)")
    ap.add_argument("--n-steps", type=int, default=None, help="override T (testing only)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB (a plain copy kernel of known size, "
                         "the reference for HBM counter scaling)")
    args = ap.parse_args()
    if args.main_only:
        args.no_cpu = args.no_plain = args.no_batch = args.no_serve = args.no_3d = args.no_sweep = True
        args.no_cyl = True
        args.no_precision = True
        if args.with_3d:
            args.no_3d = False
    if args.cyl_only or args.serve_mixed or args.open_only:
        args.no_cpu = True
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding the channels over "
              "several GPUs is not built.", file=sys.stderr)
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
        if not args.no_cyl and not args.cyl_only:
            cpu["reduced"] = cpu_baseline_reduced()
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
    if args.c4_full:
        nw = args.c4_full_waves or (3 if args.c4_full_precision == "fp32" else 16)
        run = range(args.c4_full_from, nw if not args.c4_full_count else
                    min(nw, args.c4_full_from + args.c4_full_count))
        print(json.dumps(bench_3d_full(cf, torch, waves=nw, precision=args.c4_full_precision, run=run)),
              flush=True)
        return
    if args.serve_mixed:
        print(json.dumps(bench_serving_mixed(cf, torch, args)), flush=True)
        return
    if args.open_only:
        print(json.dumps(bench_open_space(cf, torch)), flush=True)
        return
    if args.cyl_only:
        rec = bench_cyl(cf, torch, quick=args.cyl_quick)
        if not args.cyl_quick:
            rec["kz"] = bench_kz(cf, torch)
        print(json.dumps(rec), flush=True)
        return
    prob = cf.Problem.from_workload(wl)
    opts = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol=wl.pol,
                kernel=wl.kernel, precision="fp32", tile_variant=args.tile_variant)
    info = prob.info(**opts)
    ws = torch.empty(info["workspace_bytes"], dtype=torch.uint8, device="cuda")
    log(f"[bench] {wl.name}: {info['n_channels']} channels, {wl.n_cells} cells, T={wl.n_steps}, "
        f"workspace {info['workspace_bytes'] / 2**20:.1f} MiB")

    if args.stencil_only:
        rt = prob.solve(workspace=ws, time_stencil=True, **opts)
        print(json.dumps({"workload": wl.name, "tile_variant": rt["tile_variant"],
                          "avg_launch_ms": rt["stencil_ms_avg"], "launches_timed": rt["stencil_samples"],
                          "launches": rt["stencil_launches"], "device_ms": rt["device_ms"]}), flush=True)
        return
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
        log(f"[bench] step {k}: {lat[-1]:.1f} ms (device {r['device_ms']:.1f} ms) force {r['force']:.10e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cu_per_solve = r["cell_updates"]
    value = cu_per_solve * args.steps / elapsed

    # dominant kernel: field update, timed live with HIP events on the solve's stream
    rt = prob.solve(workspace=ws, time_stencil=True, **opts)
    avg_s = rt["stencil_ms_avg"] * 1e-3
    alg_bytes = rt["stencil_alg_bytes"]
    # cells the kernel advances per launch (waves holding only conductor skipped)
    adv_cells = rt["stencil_cell_updates"] * rt["advanced_cell_updates"] / rt["cell_updates"]
    traffic, traffic_note = measured_traffic(rt["tile_variant"])
    valu, valu_note = measured_valu(rt["tile_variant"])
    # The kernel keeps several steps per launch in registers and skips rows of
    # conductor, so its algorithmic bytes exceed what HBM could deliver in the
    # launch time: the binding resource is vector-instruction issue (VALU),
    # reported against the issue ceiling with the counter record's
    # instructions per launch and the live launch time.
    roofline = {"bound": "alu",
                "achieved": valu / avg_s if (valu and avg_s > 0) else None,
                "peak": VALU_PEAK_WAVE_INSTR, "unit": "VALU wave-instructions/s",
                "frac": valu / avg_s / VALU_PEAK_WAVE_INSTR if (valu and avg_s > 0) else None,
                "valu_instr_per_launch": valu, "valu_note": valu_note,
                "useful_valu_frac": (STEP_LANE_INSTR * adv_cells / 64.0) / avg_s / VALU_PEAK_WAVE_INSTR
                if avg_s > 0 else None,
                "step_lane_instr_per_cell_update": STEP_LANE_INSTR,
                "advanced_cells_per_launch": adv_cells,
                "traffic": traffic, "traffic_note": traffic_note,
                "hbm_real_frac": traffic / avg_s / (HBM_PEAK_GBS * 1e9) if (traffic and avg_s > 0) else None,
                "alg_bytes_per_launch": alg_bytes,
                "alg_bytes_per_cell_update": alg_bytes / rt["stencil_cell_updates"],
                "alg_hbm_ratio": alg_bytes / avg_s / (HBM_PEAK_GBS * 1e9) if avg_s > 0 else None,
                "kernel": "k_rb2d: fused register-blocked 2D update of all TM (or TE) channels, "
                          "steps_per_launch time steps per launch",
                "avg_launch_ms": rt["stencil_ms_avg"], "launches_timed": rt["stencil_samples"],
                "tile_variant": rt["tile_variant"], "steps_per_launch": rt["tile_halo"],
                "launches_per_solve": rt["stencil_launches"],
                # the timed solves run the TM and the TE launches on two streams, so that
                # each polarization's launch tail overlaps the other's; over a whole solve
                # the VALU issue rate is (instructions per launch x launches) / device time
                "solve_valu_frac": (valu * rt["stencil_launches"] / (r["device_ms"] * 1e-3) / VALU_PEAK_WAVE_INSTR
                                    if valu and r["device_ms"] > 0 else None),
                "solve_valu_note": "per-launch figures (frac, traffic) come from a solve whose launches run "
                                   "one at a time (launch sampling turns the two streams off)"}

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
           "force": r["force"], "roofline": roofline,
           "advanced_cell_updates_per_s": r["advanced_cell_updates"] * args.steps / elapsed,
           "device_ms_per_solve": r["device_ms"]}

    # every fused-kernel variant on the same solve (T = 1000), the autotuner's
    # search space; all variants give bitwise-identical results
    sweep = []
    for v in (range(1, 32) if not args.no_sweep else ()):
        try:
            rv = prob.solve(workspace=ws, **dict(opts, n_steps=1000, tile_variant=v))
        except cf.CfError:
            break
        if not rv["fused"] or rv["tile_variant"] != v:
            break
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rv = prob.solve(workspace=ws, **dict(opts, n_steps=1000, tile_variant=v))
        sweep.append({"variant": v, "steps_per_launch": rv["tile_halo"],
                      "ms_per_1000_steps": (time.perf_counter() - t1) * 1e3})
    out["tile_sweep"] = sweep

    if not args.no_batch:
        # batching extension: the 24-clearance uneven piston set (h in [0.1, 2],
        # grid heights 84..160) with metallic sidewalls, and the same set with
        # mu = 5 magnetic sidewalls, each in one batched, graph-captured launch
        # sequence at the full T; then one batched sequence against one fused
        # solve after another (metallic set, T = 2000)
        from casimir_inputs import c3_uneven_set
        for side, key in (("pec", "batched_uneven"), ("mu5", "batched_uneven_mu5")):
            set_wl = c3_uneven_set(side)
            T_b = set_wl[0].n_steps
            probs = [cf.Problem.from_workload(w) for w in set_wl]
            bo = dict(opts, n_steps=T_b, kernel=set_wl[0].kernel)
            cf.batch_solve(probs, graph=True, **dict(bo, n_steps=16))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rb = cf.batch_solve(probs, graph=True, **bo)
            tb = time.perf_counter() - t1
            cu = sum(r["cell_updates"] for r in rb)
            walls = "metallic" if side == "pec" else "mu = 5 magnetic"
            out[key] = {"workload": f"24 TE+TM pistons, h = linspace(0.1, 2.0), 400 x (84..160), {walls} sidewalls, "
                                    f"{sum(r['n_channels'] for r in rb)} channels, T={T_b}, FP32, one graph-captured "
                                    "batched sequence",
                        "value": cu / tb, "unit": "cell-updates/s", "ms": tb * 1e3,
                        "fused_problems": sum(1 for r in rb if r["fused"]),
                        "tile_variants": sorted({r["tile_variant"] for r in rb})}
            log(f"[bench] batched {side}: 24 problems, T={T_b}: {tb * 1e3:.0f} ms ({cu / tb:.3e} cell-updates/s)")
        T_s = 2000
        probs = [cf.Problem.from_workload(w.replace(n_steps=T_s)) for w in c3_uneven_set("pec")]
        bo = dict(opts, n_steps=T_s)
        cf.batch_solve(probs, graph=True, **bo)
        for p_ in probs:
            p_.solve(**bo)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cf.batch_solve(probs, graph=True, **bo)
        tb = time.perf_counter() - t1
        t1 = time.perf_counter()
        for p_ in probs:
            p_.solve(**bo)
        ts = time.perf_counter() - t1
        out["batched_uneven"].update({"vs_sequential": {"T": T_s, "batched_ms": tb * 1e3, "sequential_ms": ts * 1e3,
                                                        "speedup": ts / tb}})
        log(f"[bench] batched vs one after another (T={T_s}): {tb * 1e3:.0f} ms vs {ts * 1e3:.0f} ms")

    rate_3d = None
    if not args.no_3d:
        out["c4_3d"] = bench_3d(cf, torch, n_steps=args.c4_steps, variant=args.c4_variant)
        rate_3d = out["c4_3d"]["value"]
    if not args.no_serve:
        out["serving"] = bench_serving(cf, torch, args, rate_3d)
    if not args.no_cyl:
        out["cylindrical"] = bench_cyl(cf, torch)
        out["kz"] = bench_kz(cf, torch)

    gold = os.path.join(ROOT, "tests", "golden", "c2_piston_tetm_oracle.json")
    if os.path.exists(gold) and not args.n_steps:
        ref = json.load(open(gold))
        out["force_rel_err_vs_fp64_oracle"] = abs(r["force"] / ref["force"] - 1)
    if not args.no_precision:
        out["precision"] = bench_precision(cf, torch)

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
