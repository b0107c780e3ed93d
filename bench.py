"""Benchmark of the gridding + imaging hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-batched]

Headline workload (synthetic, seeded): the MWA-scale configuration - 512 antennas (density
~ 1/r within 1.5 km), 130,816 baselines x 32 channels x 8 times x 4 polarisations =
133,955,584 complex64 visibilities from 1000 power-law point sources; 2048^2 grid per
polarisation; prolate kernel support 7, oversampling 8; FP32 accumulation.

A step is one forward pass of the imaging hot path over the batch: mw_grid (the gridder
and its merge pass, which writes every cell, so no zeroing pass) then mw_image (+1, with
the convolution correction). The plan (FP64 positions, tile sort, work list, kernel tables)
is built once beforehand for these uvw and timed separately. Reported beside the step:
the gridder kernel alone (HIP events the library records around its own launch), a
forward + backward pass (adding the image adjoint and the degridder), and the batched
workload: 96 uneven single-polarisation jobs gridded and degridded by one multi-instance
plan (persistent launch replayed from a hipGraph) against 96 single-instance plans called
one after another. One JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mvis/s gridded (support 7, 2048² grid) + % HBM roofline; fwd+bwd vs plain"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, published
KERNEL_NAMES = {1: "k_grid_taplanes", 2: "k_grid_collanes", 3: "k_grid_scatter",
                4: "k_grid_wavetiles", 5: "k_grid_stack"}

# HBM traffic of one launch of the default gridder on this workload, from two rocprofv3
# counter passes over this script (profiles/k_grid_wavetiles_mwa2048.md): FETCH_SIZE scaled
# by 2.0 plus WRITE_SIZE scaled by 1.0, the factors a plain 1 GiB device copy reads on the
# same counters. It describes the gridder sources it was taken on (SHA-256 over the files
# below) and is reported only while they are unchanged.
GRIDDER_SOURCES = ("paper_0902_0915_amd/csrc/gridder_core.h", "paper_0902_0915_amd/csrc/grid.hip",
                   "paper_0902_0915_amd/csrc/plan.hip", "paper_0902_0915_amd/csrc/internal.h")
MEASURED_TRAFFIC = {
    "sha256": "6cfcd59d58b6a0f055264884a8ae66097b42f8ee5a37827a63a947e60076a67f",
    "fetch_kib": 1.80435e6, "write_kib": 1.74331e5, "fetch_scale": 2.0, "write_scale": 1.0,
    "profile": "profiles/k_grid_wavetiles_mwa2048.md",
}


def gridder_traffic():
    """Measured bytes per gridder launch, or None if the sources changed since."""
    import hashlib
    h = hashlib.sha256()
    for f in GRIDDER_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    m = MEASURED_TRAFFIC
    if h.hexdigest() != m["sha256"]:
        return None
    return int((m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"]) * 1024)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the kernel-stack and differentiable workloads")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="visibility groups (of 4 pols) in the oracle's timed sample "
                         "(0 = the whole workload, about 10 s on 16 host cores)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration) and exit")
    for k in ("tile", "split", "wg-waves", "flush", "order", "variant", "schedule", "autotune"):
        ap.add_argument(f"--{k}", type=int, default=0)
    return ap.parse_args()


def timed(fn, steps, stream):
    """Mean event time and mean wall time per call of fn over ``steps`` back-to-back calls."""
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall * 1e3 / steps


def percentiles(fn, steps, stream):
    """Per-call event times of fn (each call bracketed by its own events, still back to back
    on the stream): median, p10 and p90 in ms."""
    import numpy as np
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(steps):
        fn()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    t = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    return {"median": round(float(np.median(t)), 4), "p10": round(float(np.percentile(t, 10)), 4),
            "p90": round(float(np.percentile(t, 90)), 4), "n": steps}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding the "
              "work over several GPUs is not built.", file=sys.stderr)
        sys.exit(2)
    import torch

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.copy_probe:
        n = 1 << 28  # 2^28 floats = 1 GiB
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n,
                          "launches": 3}))
        return

    from paper_0902_0915_amd import mwagrid, synth

    t0 = time.perf_counter()
    log("generating the MWA-scale workload (uvw, 1000-source sky, visibilities on device)")
    wl = synth.mwa_scale(device="cuda")
    vis = wl.vis
    torch.cuda.synchronize()
    log(f"generated {wl.ngroups} groups x {wl.npol} pols in {time.perf_counter() - t0:.1f} s")

    tuning = {k: v for k, v in dict(tile=args.tile, split=args.split, wg_waves=args.wg_waves,
                                     flush=args.flush, order=args.order, variant=args.variant,
                                     schedule=args.schedule, autotune=args.autotune).items() if v}
    spec = mwagrid.InstanceSpec.from_workload(wl, with_ants=False)
    t0 = time.perf_counter()
    plan = mwagrid.Plan(spec, tuning=tuning or None)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    info = plan.info(0)
    log(f"plan built in {plan_ms:.1f} ms: {info}")

    grid = torch.empty((wl.npol, wl.ny, wl.nx), dtype=torch.complex64, device="cuda")
    img = torch.empty_like(grid)
    gback = torch.empty_like(grid)
    vout = torch.empty_like(vis)

    def step():
        plan.grid(vis, out=grid)
        plan.image(grid, direction=1, correct=True, out=img)

    def fwd_bwd():
        plan.grid(vis, out=grid)
        plan.image(grid, direction=1, correct=True, out=img)
        plan.image(img, direction=-1, correct=True, out=gback)
        plan.degrid(gback, out=vout)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps); timing {args.steps} steps")
    ev_ms, wall_ms = timed(step, args.steps, stream)
    log(f"step: {ev_ms:.3f} ms (events), {wall_ms:.3f} ms (wall)")
    step_pct = percentiles(step, args.steps, stream)
    log(f"step percentiles: {step_pct}")
    fb_ms, _ = timed(fwd_bwd, max(1, args.steps // 2), stream)
    log(f"forward + backward: {fb_ms:.3f} ms")
    # dominant kernel: the library's events around its own gridder launch, on its stream
    plan.set_timing(True)
    kms, mms = [], []
    for _ in range(args.steps):
        plan.grid(vis, out=grid)
        g, m = plan.kernel_ms(0)
        kms.append(g)
        mms.append(m)
    plan.set_timing(False)
    kern_ms = sum(kms) / len(kms)
    merge_ms = sum(mms) / len(mms)
    log(f"gridder kernel {kern_ms:.4f} ms, merge {merge_ms:.4f} ms (averages of {len(kms)})")

    nvis = info["nkept"] * wl.npol
    value = nvis / (wall_ms * 1e-3) / 1e6
    # Dominant kernel: the gridder. Its algorithmic bytes are the kept visibilities, each read
    # once (8 B per polarisation); the grid write (8 B per cell per polarisation) belongs to
    # the merge launch, and both together make one mw_grid call.
    kname = f"{KERNEL_NAMES.get(info['variant'], 'k_grid')}<{wl.npol},{wl.W}>"
    alg_bytes_kernel = nvis * 8
    kern_gbs = alg_bytes_kernel / (kern_ms * 1e-3) / 1e9
    traffic = gridder_traffic() if (info["variant"] == 4 and info["flush"] == 2 and not tuning) else None
    roofline = {"bound": "hbm", "achieved": round(kern_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(kern_gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
                "kernel_ms": round(kern_ms, 4), "alg_bytes_per_launch": alg_bytes_kernel,
                "traffic_profile": MEASURED_TRAFFIC["profile"] if traffic else None}
    # The whole mw_grid call (gridder + merge) against HBM, and the step.
    alg_bytes = nvis * 8 + wl.npol * wl.nx * wl.ny * 8
    step_gbs = alg_bytes / (wall_ms * 1e-3) / 1e9
    grid_gbs = alg_bytes / ((kern_ms + merge_ms) * 1e-3) / 1e9
    hbm = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s", "alg_bytes_per_grid": alg_bytes,
           "gridding_achieved": round(grid_gbs, 1), "gridding_frac": round(grid_gbs / HBM_PEAK_GBS, 4),
           "step_frac": round(step_gbs / HBM_PEAK_GBS, 4)}
    # The same kernel against the FP32 vector peak: 49 taps x npol x complex-by-real FMA
    # (4 flop) per kept group, the direct form's count.
    alg_flop = info["nkept"] * wl.W * wl.W * wl.npol * 4
    tflops = alg_flop / (kern_ms * 1e-3) / 1e12
    alu = {"bound": "alu", "achieved": round(tflops, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
           "unit": "TFLOP/s", "frac": round(tflops / FP32_VECTOR_PEAK_TFLOPS, 4),
           "alg_flop_per_launch": alg_flop}

    # Stokes conversion of the step's four corrected images with a per-pixel instrument
    # response (2048^2): reads 32 B of images and 32 B of Jones matrix per pixel, writes 16 B.
    jones = torch.from_numpy(synth.jones_field(wl.nx, wl.ny, hour_angle=0.1)).cuda()
    stokes_out = torch.empty((4, wl.ny, wl.nx), dtype=torch.float32, device="cuda")
    plan.stokes(img, jones, out=stokes_out)
    st_pct = percentiles(lambda: plan.stokes(img, jones, out=stokes_out), args.steps, stream)
    st_bytes = wl.nx * wl.ny * (32 + 32 + 16)
    stokes = {"workload": f"{wl.ny}x{wl.nx} pixels x 4 polarisations, per-pixel Jones matrices",
              "ms": st_pct, "alg_bytes": st_bytes,
              "achieved_gbs": round(st_bytes / (st_pct["median"] * 1e-3) / 1e9, 1),
              "frac_hbm": round(st_bytes / (st_pct["median"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    log(f"stokes: {stokes}")
    del jones, stokes_out

    # Plan for new uvw (a new snapshot) plus one grid call.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with mwagrid.Plan(spec, tuning=tuning or None) as p2:
        p2.grid(vis, out=grid)
        torch.cuda.synchronize()
        plan_grid_ms = (time.perf_counter() - t0) * 1e3
    log(f"plan + one grid: {plan_grid_ms:.1f} ms")

    cml = None if args.no_extra else bench_calibration(mwagrid, wl, stream)
    stacks = None if args.no_extra else bench_stacks(mwagrid, synth, stream, args.steps)
    diff = None if args.no_extra else bench_differentiable(mwagrid, synth, stream, args.steps)

    batched = None
    if not args.no_batched:
        batched = bench_batched(mwagrid, synth, stream, max(3, args.steps // 4))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, vis, args.cpu_sample)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mvis/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mwa_scale: 512 antennas (1/r density, 1.5 km), 130816 baselines"
                               " x 32 channels x 8 times x 4 pols, 1000 sources, 2048^2 grid,"
                               " W=7, O=8", "visibilities": nvis, "grid": [wl.npol, wl.ny, wl.nx],
                   "launch": {k: info[k] for k in ("tile", "split", "wg_waves", "order",
                                                   "variant", "flush", "schedule", "nwork")}},
        "roofline": roofline,
        "grid_call_roofline": hbm,
        "alu_roofline": alu,
        "grid_mvis_s": round(nvis / ((kern_ms + merge_ms) * 1e-3) / 1e6, 1),
        "merge_ms": round(merge_ms, 4),
        "step_event_ms": round(ev_ms, 4),
        "step_ms_percentiles": step_pct,
        "plan_ms": round(plan_ms, 1),
        "plan_plus_grid_ms": round(plan_grid_ms, 1),
        "fwd_bwd_ms": round(fb_ms, 4),
        "stokes": stokes,
        "calibration": cml,
        "kernel_stacks": stacks,
        "differentiable": diff,
        "batched": batched,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    plan.close()


def bench_calibration(mwagrid, wl, stream):
    """The calibration measurement loop on the MWA-scale visibilities: the 20 brightest
    sources of the workload's own sky peeled in decreasing flux, 10 StEFCal iterations each
    (per source: one pass forming per-row sums against its prediction, the iterations over
    the rows' sums, one pass removing it), and the prediction of all 1000 sources."""
    import numpy as np
    import torch
    spec = mwagrid.InstanceSpec.from_workload(wl, with_ants=True)
    plan = mwagrid.Plan(spec)
    sky = np.stack([wl.sky.l, wl.sky.m, wl.sky.flux], axis=1)
    cat = sky[np.argsort(-sky[:, 2], kind="stable")[:20]]
    plan.peel(wl.vis, cat, niter=10)
    peel = percentiles(lambda: plan.peel(wl.vis, cat, niter=10), 5, stream)
    src = torch.from_numpy(sky).cuda()
    out = torch.empty_like(wl.vis)
    plan.predict(src, out=out)
    pred = percentiles(lambda: plan.predict(src, out=out), 3, stream)
    plan.close()
    terms = wl.ngroups * sky.shape[0]
    res = {"workload": "mwa_scale visibilities (512 antennas, 4 pols), 20 brightest of the 1000-source sky",
           "peel_ms": peel, "per_source_ms": round(peel["median"] / 20, 4), "niter": 10,
           "predict_1000_sources_ms": pred,
           "predict_gterms_s": round(terms / (pred["median"] * 1e-3) / 1e9, 2)}
    log(f"calibration: {res}")
    return res


def bench_stacks(mwagrid, synth, stream, steps):
    """Kernel stacks (128 antennas x 8 channels x 16 times, 4096^2 grid, O = 4, A-term x
    w-plane kernels of support 21...45): grid and degrid times. This workload is bound by
    LDS and VALU work on the taps, not by HBM: it is reported against the FP32 vector peak
    with 8 flop per tap (a complex tap times a complex visibility, added: 4 FMAs)."""
    import numpy as np
    import torch
    wl = synth.beam_w_stacks()
    spec = mwagrid.InstanceSpec.from_workload(wl, with_ants=False)
    t0 = time.perf_counter()
    plan = mwagrid.Plan(spec)
    torch.cuda.synchronize()
    pms = (time.perf_counter() - t0) * 1e3
    vis = torch.from_numpy(wl.vis).cuda()
    grid = torch.empty((1, wl.ny, wl.nx), dtype=torch.complex64, device="cuda")
    vout = torch.empty_like(vis)
    plan.grid(vis, out=grid)
    plan.degrid(grid, out=vout)
    g = percentiles(lambda: plan.grid(vis, out=grid), steps, stream)
    d = percentiles(lambda: plan.degrid(grid, out=vout), steps, stream)
    info = plan.info(0)
    plan.close()
    sel = wl.kernel_index if wl.flags is None else wl.kernel_index[wl.flags == 0]
    sup = wl.kernel_support[sel].astype(np.int64)
    taps = int((sup * sup).sum())
    flop = 8 * taps  # complex x complex multiply-add per tap
    out = {"workload": "beam_w_stacks: 128 antennas x 8 ch x 16 times, 4096^2, O=4, supports 21..45",
           "visibilities": int(info["nkept"]), "taps": taps, "plan_ms": round(pms, 1),
           "grid_ms": g, "degrid_ms": d,
           "grid_mvis_s": round(info["nkept"] / (g["median"] * 1e-3) / 1e6, 1),
           "grid_tflops": round(flop / (g["median"] * 1e-3) / 1e12, 2),
           "grid_frac_fp32_vector": round(flop / (g["median"] * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS, 4),
           # every tap is a complex64 gathered from the kernel stack: its read rate
           "grid_tap_read_gbs": round(8 * taps / (g["median"] * 1e-3) / 1e9, 1),
           "launch": {k: info[k] for k in ("tile", "variant", "wg_waves", "nwork")}}
    log(f"kernel stacks: {out}")
    return out


def bench_differentiable(mwagrid, synth, stream, steps):
    """Differentiable imaging (128 antennas x 8 ch x 4 times, 1024^2): forward = gains ->
    grid -> image, loss = ||image - target||^2, backward through the hand-written adjoints to
    the visibilities and gains, as one autograd step."""
    import numpy as np
    import torch
    from paper_0902_0915_amd.mwagrid import grid_image
    wl = synth.differentiable()
    spec = mwagrid.InstanceSpec.from_workload(wl)
    plan = mwagrid.Plan(spec)
    vis = torch.from_numpy(wl.vis).cuda().requires_grad_(True)
    g = torch.from_numpy(wl.gains.astype(np.complex64)).cuda().requires_grad_(True)
    with torch.no_grad():
        target = grid_image(vis.detach(), None, plan, correct=False).clone()

    def step():
        vis.grad = None
        g.grad = None
        img = grid_image(vis, g, plan, correct=False)
        loss = torch.sum(torch.abs(img - target) ** 2)
        loss.backward()

    for _ in range(3):
        step()
    pct = percentiles(step, steps, stream)
    plan.close()
    out = {"workload": "differentiable: 128 antennas x 8 ch x 4 times, 1024^2, gains",
           "visibilities": wl.ngroups, "fwd_bwd_ms": pct,
           "steps_per_s": round(1e3 / pct["median"], 1)}
    log(f"differentiable: {out}")
    return out


def bench_batched(mwagrid, synth, stream, steps):
    """96 uneven jobs: one batched plan (persistent launch + graph replay) against 96
    single-instance plans, forward (grid) + backward (degrid) each."""
    import torch

    t0 = time.perf_counter()
    log("batched workload: generating 96 uneven jobs")
    jobs = synth.batched_jobs(device="cuda")
    torch.cuda.synchronize()
    nvis = sum(int((j.flags == 0).sum()) for j in jobs)
    log(f"batched workload: {nvis} kept visibilities in {time.perf_counter() - t0:.1f} s")
    specs = [mwagrid.InstanceSpec.from_workload(j, with_ants=False) for j in jobs]
    vis = [j.vis for j in jobs]
    # the plan is built three times: the first in the process pays one-time costs (kernel
    # tables of new sizes, pool blocks, worker threads); a pipeline re-planning every snapshot
    # pays the later ones
    plan_ms = []
    for rep in range(3):
        t0 = time.perf_counter()
        bplan = mwagrid.Plan(specs)
        torch.cuda.synchronize()
        plan_ms.append((time.perf_counter() - t0) * 1e3)
        if rep < 2:
            bplan.close()
    bplan_ms = plan_ms[0]
    log(f"batched plan: {plan_ms[0]:.1f} ms first, {min(plan_ms[1:]):.1f} ms rebuilt")
    grids = bplan.new_grids()
    vouts = [torch.empty_like(v) for v in vis]

    def batched_step():
        bplan.grid(vis, out=grids)
        bplan.degrid(grids, out=vouts)

    singles = [mwagrid.Plan(sp) for sp in specs]

    def sequential_step():
        for p, v, g, o in zip(singles, vis, grids, vouts):
            p.grid(v, out=g)
            p.degrid(g, out=o)

    for _ in range(2):
        batched_step()
        sequential_step()
    b_ms, _ = timed(batched_step, steps, stream)
    s_ms, _ = timed(sequential_step, steps, stream)
    log(f"batched fwd+bwd {b_ms:.3f} ms vs sequential {s_ms:.3f} ms")
    for p in singles:
        p.close()
    bplan.close()
    return {"workload": "96 jobs, kept visibilities logU[1e4, 2e6] after 5-30% flagging, "
                        "grids {512..4096}^2, W=7, O=8, 1 pol",
            "visibilities": nvis, "batched_fwd_bwd_ms": round(b_ms, 4),
            "sequential_fwd_bwd_ms": round(s_ms, 4), "speedup": round(s_ms / b_ms, 3),
            "batched_mvis_s": round(nvis / (b_ms * 1e-3) / 1e6, 1),
            "sequential_mvis_s": round(nvis / (s_ms * 1e-3) / 1e6, 1),
            "batched_plan_ms": round(bplan_ms, 1), "batched_replan_ms": round(min(plan_ms[1:]), 1)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, vis_dev, sample_groups):
    """The FP64 oracle (as it stands) on the same workload, or its first ``sample_groups``
    groups: positions, gridding (all host cores, row stripes) and the image with
    correction; scaled to Mvis/s."""
    import oracle as orc

    ng = min(sample_groups, wl.ngroups) if sample_groups > 0 else wl.ngroups
    nrow = ng // wl.nchan
    ng = nrow * wl.nchan
    cores = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        cores = min(cores, int(os.environ["OMP_NUM_THREADS"]))
    log(f"cpu baseline: oracle on {ng} groups ({nrow} rows) with {cores} threads")
    vis = vis_dev[:ng].cpu().numpy()
    # whole passes until about 10 s of CPU work (at most 8)
    passes, total = 0, 0.0
    while passes < 8 and (passes == 0 or total < 10.0):
        t0 = time.perf_counter()
        pos, keep, _ = orc.positions(wl.uvw[:nrow], wl.freq, wl.nx, wl.ny, wl.du, wl.dv, wl.W, wl.O)
        G = orc.grid(pos, keep, vis, wl.nx, wl.ny, wl.W, wl.O, nchan=wl.nchan, nthreads=cores)
        orc.image(G, W=wl.W, correct=True)
        total += time.perf_counter() - t0
        passes += 1
    dt = total / passes
    nv = int(keep.sum()) * wl.npol
    log(f"cpu baseline: {passes} passes, {dt:.2f} s each")
    # one core, on the first sixteenth of the rows (the same per-visibility work)
    nrow1 = max(1, nrow // 16)
    ng1 = nrow1 * wl.nchan
    vis1 = vis[:ng1]
    t1, p1 = 0.0, 0
    while p1 < 4 and (p1 == 0 or t1 < 8.0):
        t0 = time.perf_counter()
        pos, keep1, _ = orc.positions(wl.uvw[:nrow1], wl.freq, wl.nx, wl.ny, wl.du, wl.dv, wl.W, wl.O)
        G = orc.grid(pos, keep1, vis1, wl.nx, wl.ny, wl.W, wl.O, nchan=wl.nchan, nthreads=1)
        orc.image(G, W=wl.W, correct=True)
        t1 += time.perf_counter() - t0
        p1 += 1
    nv1 = int(keep1.sum()) * wl.npol
    log(f"cpu baseline, one core: {p1} passes, {t1 / p1:.2f} s each")
    return {"value": round(nv / dt / 1e6, 3), "unit": "Mvis/s", "cores": cores,
            "kind": "oracle", "seconds": round(total, 2), "passes": passes, "cpu_model": cpu_model(),
            "sample": (f"the whole workload ({nv} kept visibilities)" if nrow == wl.uvw.shape[0] else
                       f"first {nrow} rows x {wl.nchan} channels x {wl.npol} pols of the same "
                       f"workload ({nv} visibilities)")
                      + f", positions + grid + corrected image, mean of {passes} passes",
            "single_core": {"value": round(nv1 / (t1 / p1) / 1e6, 3), "unit": "Mvis/s", "cores": 1,
                            "seconds": round(t1, 2), "passes": p1,
                            "sample": f"first {nrow1} rows x {wl.nchan} channels x {wl.npol} pols "
                                      f"({nv1} visibilities), positions + grid + corrected image "
                                      "(the 2048^2 image transform included in each pass)"}}


if __name__ == "__main__":
    main()
