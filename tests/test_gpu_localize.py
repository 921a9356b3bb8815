"""GPU parity of the localisation loop (Sec. III-C: variance-triggered
refinement stages) and of its two new pieces, the position variance and the
full-image render, against the FP64 oracle.

The loop is checked in lockstep: the library records every iteration's
predicted poses, weights and drawn indices (loc_trace); at each iteration the
oracle weights the same input set and must agree within the FP32 update's
tolerances, while every decision that floating point turns into an integer
(the stage switch, the drawn indices) is re-taken by the oracle from the
library's own float64 values and must agree exactly.

Tolerances: poses 1e-12 (float64 both sides); variance and read-out of the
library's weighted set 1e-12 relative (float64 both sides, different
summation order); render C, A as the small map's update parity (2e-5) and the
8x256 map's (2e-4); weights 1e-2 relative above 1e-6 and 1e-6 absolute below
(the small map's update tolerance).
"""
import math

import numpy as np
import pytest

from oracle import mcl, se3
from oracle import render as rd
from paper_2406_12202_amd import synth
from parity_util import stats

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _ctx(spec, params, precision="fp32"):
    from paper_2406_12202_amd import binding
    return binding.Context(spec, params, precision=precision)


# ------------------------------------------------------------ position variance

@pytest.mark.parametrize("N", [1, 7, 256, 1000, 4099])
def test_position_variance_matches_oracle(torch_dev, N):
    torch = torch_dev
    rng = np.random.default_rng([N, 11])
    P = synth.particles("small", 3, N=N)
    P[:, :, 3] += rng.normal(0.0, 0.3, (N, 3))
    w = rng.exponential(1.0, N)
    if N > 4:
        w[rng.choice(N, N // 4, replace=False)] = 0.0
        w[1] = -0.5
        w[2] = np.nan
        w[3] = np.inf
    ctx = _ctx(synth.spec("small"), synth.map_params(synth.spec("small"), 3))
    dev = torch.device("cuda", 0)
    var = ctx.loc_position_variance(torch.as_tensor(P, device=dev).contiguous(), torch.as_tensor(w, device=dev))
    got = float(var.cpu().numpy()[0])
    want = mcl.position_variance(P, w)
    print("N=%d var gpu=%.17g oracle=%.17g" % (N, got, want), flush=True)
    if N == 1:
        assert got == 0.0 and want == 0.0
    else:
        assert abs(got - want) <= 1e-12 * abs(want)
    ctx.close()


def test_position_variance_without_weight_is_nan(torch_dev):
    torch = torch_dev
    P = synth.particles("small", 4, N=16)
    dev = torch.device("cuda", 0)
    ctx = _ctx(synth.spec("small"), synth.map_params(synth.spec("small"), 4))
    for w in (np.zeros(16), np.full(16, -1.0), np.full(16, np.nan)):
        var = ctx.loc_position_variance(torch.as_tensor(P, device=dev).contiguous(), torch.as_tensor(w, device=dev))
        assert math.isnan(float(var.cpu().numpy()[0]))
        assert math.isnan(mcl.position_variance(P, w))
    ctx.close()


# ------------------------------------------------------------------ render image

def _oracle_pixels(spec, params, pose, cam, inv_R, pix, seed, it):
    W, H, fx, fy, cx, cy = cam
    Wl = W // inv_R
    P = rd.unpack(spec, params)
    rays = mcl.particle_rays(pose, pix, Wl, (fx / inv_R, fy / inv_R, cx / inv_R, cy / inv_R))
    return mcl.render_rays(spec, P, rays, [(0, p) for p in pix], seed, it)


@pytest.mark.parametrize("inv_R", [1, 2])
def test_render_image_small_map_every_pixel(torch_dev, inv_R):
    torch = torch_dev
    spec = synth.spec("small")
    params = synth.map_params(spec, 5)
    cam = (48, 40, 45.0, 45.0, 24.0, 20.0)
    pose = synth.gt_pose("small", 5)
    dev = torch.device("cuda", 0)
    ctx = _ctx(spec, params)
    rgb, op = ctx.loc_render_image(cam, inv_R, torch.as_tensor(pose, device=dev).contiguous(), seed=9, iter=2,
                                   opacity=True)
    rgb, op = rgb.cpu().numpy().astype(np.float64), op.cpu().numpy().astype(np.float64)
    Hl, Wl = cam[1] // inv_R, cam[0] // inv_R
    assert rgb.shape == (Hl, Wl, 3) and op.shape == (Hl, Wl)
    pix = list(range(Wl * Hl))
    r = _oracle_pixels(spec, params, pose, cam, inv_R, pix, 9, 2)
    rc = stats("C", rgb.reshape(-1, 3), r["C"])
    ra = stats("A", op.reshape(-1), r["A"])
    assert rc["max"] <= 2e-5 and ra["max"] <= 2e-5
    ctx.close()


def test_render_image_nerf_map_hierarchical_sampled(torch_dev):
    torch = torch_dev
    spec = synth.spec("nerf")
    params = synth.map_params(spec, 6)
    cam = synth.camera("nerf")
    pose = synth.gt_pose("nerf", 6)
    inv_R = 4
    dev = torch.device("cuda", 0)
    ctx = _ctx(spec, params)
    rgb = ctx.loc_render_image(cam, inv_R, torch.as_tensor(pose, device=dev).contiguous(), seed=3, iter=1)
    rgb = rgb.cpu().numpy().astype(np.float64)
    Wl, Hl = cam[0] // inv_R, cam[1] // inv_R
    rng = np.random.default_rng(6)
    pix = sorted(set(rng.choice(Wl * Hl, 48, replace=False).tolist()) | {0, Wl * Hl - 1})
    r = _oracle_pixels(spec, params, pose, cam, inv_R, pix, 3, 1)
    rc = stats("C", rgb.reshape(-1, 3)[pix], r["C"])
    assert rc["max"] <= 2e-4
    ctx.close()


def test_render_image_rejects_bad_level(torch_dev):
    torch = torch_dev
    from paper_2406_12202_amd.binding import LocError
    spec = synth.spec("small")
    ctx = _ctx(spec, synth.map_params(spec, 7))
    pose = torch.as_tensor(synth.gt_pose("small", 7), device=torch.device("cuda", 0)).contiguous()
    with pytest.raises(LocError):
        ctx.loc_render_image((50, 40, 45.0, 45.0, 25.0, 20.0), 4, pose)
    with pytest.raises(LocError):
        ctx.loc_render_image((48, 40, 45.0, 45.0, 24.0, 20.0), 3, pose)
    ctx.close()


# ------------------------------------------------------------ localisation loop

def _check_lockstep(spec, params, img, cam, stages, poses0, out, seed, sigma_t, sigma_r, motion=None):
    """Walk the library's trace iteration by iteration against the oracle."""
    steps = out["steps"]
    tp = out["trace"]["pose"].cpu().numpy()
    tw = out["trace"]["weight"].cpu().numpy()
    ti = out["trace"]["idx"].cpu().numpy()
    X = np.asarray(poses0, dtype=np.float64)
    s = 0
    toff = ioff = 0
    for t, rec in enumerate(steps):
        inv_R, B = stages[s][:2]
        kn = stages[s][4] if len(stages[s]) > 4 else 1.0
        assert rec["iter"] == t and rec["stage"] == s and rec["n"] == X.shape[0]
        n = rec["n"]
        o = mcl.update_particles(spec, params, img, cam, inv_R, B, X, motion, kn * sigma_t, kn * sigma_r, seed, t)
        pred, w = tp[toff:toff + n], tw[toff:toff + n]
        assert np.allclose(pred.reshape(n, 12), o["pose"].reshape(n, 12), atol=1e-12, rtol=0)
        big = o["weight"] > 1e-6
        rw = np.abs(w - o["weight"])[big] / o["weight"][big]
        print("t=%d stage=%d n=%d var=%.6g max rel w=%.3e" % (t, s, n, rec["var"], rw.max() if rw.size else 0.0),
              flush=True)
        assert rw.size == 0 or rw.max() <= 1e-2
        assert np.all(np.abs(w - o["weight"])[~big] <= 1e-6)
        # read-outs of the library's own weighted set
        v = mcl.position_variance(pred, w)
        assert abs(rec["var"] - v) <= 1e-12 * abs(v)
        e = se3.pose_estimate(pred, w)
        assert np.allclose(rec["est"], e, atol=1e-12, rtol=0)
        # stage switch and draw, re-taken from the library's values
        if s + 1 < len(stages) and rec["var"] < stages[s][3]:
            s += 1
        n_next = stages[s][2]
        assert rec["n_next"] == n_next
        idx = mcl.resample(w, n_next, seed, t)
        assert idx is not None
        assert np.array_equal(ti[ioff:ioff + n_next], np.asarray(idx, dtype=np.int32))
        X = pred[np.asarray(idx)]
        toff += n
        ioff += n_next
    return X, s


def _small_case(seed):
    spec = synth.spec("small")
    params = synth.map_params(spec, seed)
    cam = synth.camera("small")
    img = synth.observation("small", seed)
    poses = synth.particles("small", seed, N=40)
    return spec, params, cam, img, poses


def test_localize_lockstep_with_stage_switch(torch_dev):
    torch = torch_dev
    seed = 21
    spec, params, cam, img, poses = _small_case(seed)
    dev = torch.device("cuda", 0)
    img_d = torch.as_tensor(img, device=dev)
    pose_d = torch.as_tensor(poses, device=dev).contiguous()
    ctx = _ctx(spec, params)
    kw = dict(sigma_t=0.05, sigma_r=0.03, seed=seed)
    # never switching: delta 0 (a variance is never below 0)
    base = [(2, 8, 48, 0.0), (1, 16, 24, 0.0)]
    a = ctx.loc_localize(img_d, cam, base, 4, pose_d, trace_capacity=4 * 48, **kw)
    assert [r["stage"] for r in a["steps"]] == [0, 0, 0, 0]
    # a threshold met at the first iteration whose variance reaches the run's minimum
    k = int(np.argmin([r["var"] for r in a["steps"][:3]]))
    stages = [(2, 8, 48, a["steps"][k]["var"] * (1 + 1e-9)), (1, 16, 24, 0.0)]
    b = ctx.loc_localize(img_d, cam, stages, 5, pose_d, trace_capacity=5 * 48, **kw)
    seq = [r["stage"] for r in b["steps"]]
    print("stages", seq, flush=True)
    assert seq[:k + 1] == [0] * (k + 1) and seq[k + 1:] == [1] * (4 - k)
    for t in range(k + 1):
        assert b["steps"][t]["var"] == a["steps"][t]["var"]
    X, s = _check_lockstep(spec, params, img, cam, stages, poses, b, seed, 0.05, 0.03)
    assert s == 1
    assert b["pose"].shape[0] == 24
    assert np.array_equal(b["pose"].cpu().numpy(), X)
    ctx.close()


def test_localize_three_stages_with_motion(torch_dev):
    torch = torch_dev
    seed = 22
    spec, params, cam, img, poses = _small_case(seed)
    dev = torch.device("cuda", 0)
    motion = se3.exp_se3(np.array([0.02, 0.0, -0.01]), np.array([0.01, -0.02, 0.015]))
    ctx = _ctx(spec, params)
    stages = [(4, 4, 64, math.inf, 2.0), (2, 8, 32, math.inf), (1, 16, 16, 0.0, 0.5)]
    out = ctx.loc_localize(torch.as_tensor(img, device=dev), cam, stages, 4,
                           torch.as_tensor(poses, device=dev).contiguous(), motion=motion, sigma_t=0.02,
                           sigma_r=0.01, seed=seed, iter=0, trace_capacity=4 * 64)
    assert [r["stage"] for r in out["steps"]] == [0, 1, 2, 2]
    assert [r["n"] for r in out["steps"]] == [40, 32, 16, 16]
    X, _ = _check_lockstep(spec, params, img, cam, stages, poses, out, seed, 0.02, 0.01, motion=motion)
    assert np.array_equal(out["pose"].cpu().numpy(), X)
    ctx.close()


def test_localize_without_weight_stops(torch_dev):
    """A NaN observation gives no particle a weight: the loop
    records the iteration and stops with an empty set, as the oracle does."""
    torch = torch_dev
    seed = 23
    spec, params, cam, img, poses = _small_case(seed)
    img = np.full_like(img, np.nan)
    dev = torch.device("cuda", 0)
    ctx = _ctx(spec, params)
    stages = [(1, 8, 16, 0.0)]
    out = ctx.loc_localize(torch.as_tensor(img, device=dev), cam, stages, 3,
                           torch.as_tensor(poses, device=dev).contiguous(), seed=seed)
    assert len(out["steps"]) == 1 and out["pose"] is None
    assert out["steps"][0]["n_next"] == 0 and math.isnan(out["steps"][0]["var"])
    o = mcl.localize(spec, params, img, cam, [(1, 8, 16, 0.0)], 3, poses, seed=seed)
    assert o["pose"] is None and len(o["steps"]) == 1
    assert ctx.loc_sync() & 1
    ctx.close()


def test_localize_rejects_bad_stage(torch_dev):
    torch = torch_dev
    from paper_2406_12202_amd.binding import LocError
    spec, params, cam, img, poses = _small_case(24)
    dev = torch.device("cuda", 0)
    ctx = _ctx(spec, params)
    img_d = torch.as_tensor(img, device=dev)
    pose_d = torch.as_tensor(poses, device=dev).contiguous()
    for bad in ([(3, 8, 16, 0.0)], [(1, 0, 16, 0.0)], [(1, 8, 0, 0.0)], [(1, 8, 16, math.nan), (1, 8, 8, 0.0)],
                [(1, 8, 16, 0.0, -1.0)]):
        with pytest.raises(LocError):
            ctx.loc_localize(img_d, cam, bad, 2, pose_d)
    with pytest.raises(LocError):
        ctx.loc_localize(img_d, cam, [(1, 8, 16, 0.0)], 3, pose_d, trace_capacity=20)
    ctx.close()
