"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and the FP64 oracle on the same seeded inputs, and summarise differences."""
import math

import numpy as np

from oracle import mcl
from oracle import render as rd
from paper_2406_12202_amd import synth


def inputs(workload, seed, N=None, **spec_over):
    s = synth.spec(workload, **spec_over)
    p = synth.map_params(s, seed)
    cam = synth.camera(workload)
    poses = synth.particles(workload, seed, N=N)
    img = synth.observation(workload, seed)
    return s, p, cam, poses, img


def run_gpu(ctx, img, cam, inv_R, B, poses, motion=None, sigma_t=0.0, sigma_r=0.0, seed=0, it=0):
    import torch
    dev = torch.device("cuda", 0)
    img_d = torch.as_tensor(np.ascontiguousarray(img, dtype=np.float32), device=dev)
    pose_d = torch.as_tensor(np.ascontiguousarray(poses, dtype=np.float64), device=dev)
    po, ll, w, un = ctx.loc_update_particles(img_d, cam, inv_R, B, pose_d, motion, sigma_t, sigma_r,
                                             seed, it)
    rgb, op, F, E = ctx.loc_ray_outputs()
    flags = ctx.loc_sync()
    out = dict(pose=po.cpu().numpy(), loglik=ll.cpu().numpy(), weight=w.cpu().numpy(),
               uncert=un.cpu().numpy(), C=rgb.cpu().numpy().astype(np.float64),
               A=op.cpu().numpy().astype(np.float64), F=F.cpu().numpy().astype(np.float64),
               E=E.cpu().numpy().astype(np.float64), flags=flags)
    return out


def run_oracle(spec, params, img, cam, inv_R, B, poses, motion=None, sigma_t=0.0, sigma_r=0.0, seed=0, it=0,
               subset=None, proposal=None):
    return mcl.update_particles(spec, params, img, cam, inv_R, B, poses, motion, sigma_t, sigma_r, seed, it,
                                subset=subset, proposal=proposal)


def ctx(spec, params, precision="fp32"):
    from paper_2406_12202_amd import binding
    return binding.Context(spec, params, precision=precision)


def stats(name, a, b):
    d = np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)).ravel()
    if d.size == 0:
        return dict(name=name, n=0)
    r = dict(name=name, n=int(d.size), p50=float(np.percentile(d, 50)), p99=float(np.percentile(d, 99)),
             max=float(d.max()))
    print("%-10s n=%-7d p50=%.3e p99=%.3e max=%.3e" % (name, r["n"], r["p50"], r["p99"], r["max"]), flush=True)
    return r


def frac_over(a, b, tol):
    d = np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))
    return float((d > tol).mean())


def gt_observation(spec, params, cam, gt, B, seed, iterations, base_image, n_coarse=64, n_fine=128):
    """Observation whose query pixels for iterations 0..iterations-1 (level 1)
    hold the oracle's render of the map from pose gt (64 + 128 hierarchical
    samples, no jitter); every other pixel keeps base_image."""
    W, H, fx, fy, cx, cy = cam
    s = dict(spec, n_coarse=n_coarse, n_fine=n_fine, jitter=0)
    P = rd.unpack(s, params)
    img = np.array(base_image, dtype=np.float32, copy=True)
    pix = sorted({p for it in range(iterations) for p in mcl.pixel_indices(seed, it, B, W * H)})
    rays = mcl.particle_rays(gt, pix, W, (fx, fy, cx, cy))
    r = mcl.render_rays(s, P, rays, [(0, j) for j in range(len(pix))], 0, 0)
    for p, c in zip(pix, r["C"]):
        img[p // W, p % W] = c
    return img
