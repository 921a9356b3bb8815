#!/usr/bin/env python3
"""Throughput of the Fast Loc-NeRF particle update on one MI355X.

A step is one pass of the whole hot path over one batch: loc_update_particles
(prediction, rays, stratified + hierarchical samples, posenc + MLP,
compositing with the uncertainty F, Eq. 6 score, normalisation) followed by
loc_resample (systematic, integer-exact).  Inputs are resident in HBM before
the timed region.  Default workload: the NeRF-sized plain FP32 configuration
(8x256 map, 400 particles x 64 rays x (64 + 128) samples).

Prints one JSON line.  Per-kernel durations come from HIP events that the
library records on its own stream around every launch during the timed steps.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLP samples/s & particle updates/s, BF16+proposal vs plain FP32, 1 GPU"
PEAK = {"f32": (157.3, "TFLOP/s"), "bf16": (2500.0, "TFLOP/s"), "fp8": (5000.0, "TFLOP/s")}
HBM_PEAK = 8000.0   # GB/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="nerf", choices=["nerf", "small"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-particles", type=int, default=0,
                    help="particles of the oracle sample (default: sized to ~15 s)")
    return ap.parse_args()


def cpu_baseline(workload, spec, params, img, cam, B, poses, seed, n_particles):
    """The FP64 oracle, as it stands, timed on a bounded sample of the same
    workload; scaled to MLP samples/s."""
    from oracle import mcl
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        threads = 1
    sub = list(range(n_particles))
    t0 = time.perf_counter()
    mcl.update_particles(spec, params, img, cam, 1, B, poses, seed=seed, it=0, subset=sub)
    dt = time.perf_counter() - t0
    samples = n_particles * B * (spec["n_coarse"] + spec["n_fine"])
    return {"value": samples / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": "%d of %d particles x %d rays x (%d + %d) samples, float64 numpy, %.1f s"
                      % (n_particles, poses.shape[0], B, spec["n_coarse"], spec["n_fine"], dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the particle update is built and timed on a single MI355X; "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        return 2
    import torch
    from paper_2406_12202_amd import binding, synth

    wl = args.workload
    spec = synth.spec(wl)
    params = synth.map_params(spec, args.seed)
    cam = synth.camera(wl)
    W = synth.WORKLOADS[wl]
    N, B = W["N"], W["B"]
    poses = synth.particles(wl, args.seed)
    img = synth.observation(wl, args.seed)

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    ctx = binding.Context(spec, params, precision=args.precision, stream=stream)
    img_d = torch.as_tensor(img, device=dev)
    pose_a = torch.as_tensor(poses, device=dev).contiguous()
    pose_b = torch.empty_like(pose_a)
    ll = torch.empty(N, dtype=torch.float64, device=dev)
    w = torch.empty(N, dtype=torch.float64, device=dev)
    un = torch.empty(N, dtype=torch.float32, device=dev)
    idx = torch.empty(N, dtype=torch.int32, device=dev)

    def step(k):
        ctx.loc_update_particles(img_d, cam, 1, B, pose_a, None, 0.0, 0.0, args.seed, k,
                                 pose_out=pose_b, loglik_out=ll, weight_out=w, uncert_out=un)
        ctx.loc_resample(w, N, args.seed, k, idx_out=idx)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    ctx.loc_set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(args.steps):
        step(args.warmup + k)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    kstats = ctx.loc_kernel_stats()
    ctx.loc_set_profiling(False)
    flags = ctx.loc_sync()

    samples_per_step = N * B * (spec["n_coarse"] + spec["n_fine"])
    ms_step = ms_total / args.steps
    value = samples_per_step * args.steps / (ms_total * 1e-3)

    # dominant kernel: the map MLP (coarse and fine launches of one kernel)
    mlp = [kstats[k] for k in ("mlp_coarse", "mlp_fine") if k in kstats]
    launches = sum(m["launches"] for m in mlp)
    mlp_ms = sum(m["ms"] for m in mlp)
    mlp_flop = sum(m["flop"] for m in mlp)
    achieved = (mlp_flop / launches) / (mlp_ms / launches * 1e-3) / 1e12
    dt = "f32" if args.precision == "fp32" else "bf16"
    peak, unit = PEAK[dt]
    kname = ("k_mlp_f32" if dt == "f32" else "k_mlp_bf16") + " (%dx%d map)" % (spec["n_layers"], spec["width"])
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": None, "kernel": kname,
                "flop_per_launch": mlp_flop / launches, "avg_launch_ms": mlp_ms / launches}
    kernels = {k: {"launches": v["launches"], "avg_ms": v["ms"] / max(v["launches"], 1),
                   "share": v["ms"] / max(sum(x["ms"] for x in kstats.values()), 1e-12)}
               for k, v in kstats.items()}
    for k, v in kstats.items():
        if v["bytes"] > 0 and v["ms"] > 0:
            kernels[k]["hbm_GBps"] = v["bytes"] / (v["ms"] * 1e-3) / 1e9

    out = {"metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dt, "data": "synthetic",
           "config": {"workload": "%s: %d particles x %d rays x (%d coarse + %d fine) samples, "
                                  "%dx%d map, %dx%d image" % (wl, N, B, spec["n_coarse"], spec["n_fine"],
                                                             spec["n_layers"], spec["width"], W["W"], W["H"]),
                      "particles": N, "rays_per_particle": B, "precision": args.precision,
                      "samples_per_step": samples_per_step},
           "particle_updates_per_s": N * args.steps / (ms_total * 1e-3),
           "effective_samples_per_s": N * B * 192 * args.steps / (ms_total * 1e-3),
           "roofline": roofline, "kernels": kernels, "flags": flags, "wall_s": wall}
    if not args.no_cpu_baseline:
        n_cpu = args.cpu_particles or (48 if wl == "nerf" else 32)
        out["cpu_baseline"] = cpu_baseline(wl, spec, params, img, cam, B, poses, args.seed, n_cpu)
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
