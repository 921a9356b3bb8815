"""GPU tests of the coarse-to-fine level path (loc_update_levels: 4x64 map in
BF16, 32 samples per ray, per level a persistent fused ray kernel and a
single-workgroup level kernel, optional hipGraph replay and autotuned tiles).

* Bitwise against the unfused path: each level's per-ray results, scores and
  weights equal those of loc_update_particles + loc_resample on the same
  particles (the fused kernel repeats the unfused kernels' arithmetic).
* Against the FP64 oracle, level by level in lockstep (the oracle weights the
  GPU's own particle set of that level): predicted poses to 1e-12, per-ray
  results and l to the BF16 bars, the 1-sigma rejection decisions equal to
  the oracle's except where the mean F lies within the BF16 error of the
  threshold, the drawn indices bit-exact given the weights.
* Every tile configuration gives bitwise the same results; the autotuner's
  cache round-trips.
* Graph replays equal eager runs, with eager work and synchronisation between
  replays, over changing seeds, motion and noise.
"""
import math

import numpy as np
import pytest

from oracle import mcl
from paper_2406_12202_amd import synth
from parity_util import ctx, stats

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _dev(x, torch):
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def _setup(seed, N):
    s = synth.spec("c2f")
    p = synth.map_params(s, seed)
    cam = synth.camera("c2f")
    poses = synth.particles("c2f", seed, N=N)
    img = synth.observation("c2f", seed)
    return s, p, cam, poses, img


LEVELS_SMALL = [(4, 16, 60), (2, 24, 30), (1, 40, 12)]
MOTION = np.array([[1.0, 0.0, 0.0, 0.01], [0.0, 1.0, 0.0, -0.02], [0.0, 0.0, 1.0, 0.005]])


def _run_levels(c, img_d, cam, levels, pose_d, torch, **kw):
    po, est = c.loc_update_levels(img_d, cam, levels, pose_d, **kw)
    torch.cuda.synchronize()
    out = dict(pose=po.cpu().numpy(), est=est.cpu().numpy(), levels=[])
    for L in range(len(levels)):
        o = {k: v.cpu().numpy() for k, v in c.loc_level_outputs(L).items()}
        rgb, op, F, E = c.loc_level_ray_outputs(L)
        o.update(C=rgb.cpu().numpy(), A=op.cpu().numpy(), F=F.cpu().numpy(), E=E.cpu().numpy())
        out["levels"].append(o)
    out["flags"] = c.loc_sync()
    return out


def _same(a, b):
    return np.array_equal(a, b, equal_nan=True)


@pytest.mark.parametrize("empty_mode", [0, 1])
def test_levels_equal_unfused_path_bitwise(torch_dev, empty_mode):
    torch = torch_dev
    s, p, cam, poses, img = _setup(71, 100)
    c = ctx(s, p, "bf16")
    c.loc_set_empty_ray_uncertainty(empty_mode)
    img_d = _dev(img, torch)
    kw = dict(motion=MOTION, sigma_t=0.02, sigma_r=0.01, seed=5, iter=3)
    r = _run_levels(c, img_d, cam, LEVELS_SMALL, _dev(poses, torch), torch, reject=False, **kw)
    assert r["flags"] == 0
    u = ctx(s, p, "bf16")
    u.loc_set_empty_ray_uncertainty(empty_mode)
    X = poses
    for L, (inv_R, B, n_out) in enumerate(LEVELS_SMALL):
        po, ll, w, un = u.loc_update_particles(img_d, cam, inv_R, B, _dev(X, torch), MOTION, 0.02, 0.01, 5, 3 + L)
        rgb, op, F, E = u.loc_ray_outputs()
        idx = u.loc_resample(w, n_out, 5, 3 + L)
        g = r["levels"][L]
        assert _same(g["pose"], po.cpu().numpy()), L
        for name, ref in (("C", rgb), ("A", op), ("F", F), ("E", E), ("loglik", ll), ("weight", w), ("uncert", un),
                          ("idx", idx)):
            assert _same(g[name], ref.cpu().numpy()), (L, name)
        X = po.cpu().numpy()[idx.cpu().numpy()]
    assert _same(r["pose"], X)


# Sets that take every branch of the level kernel: level 0 has more particles
# than fit in LDS (4096) and draws more than fit there, level 1 more than fit
# but draws into LDS, level 2 fits but is too large to stage its poses in
# registers (1024) and draws more than one particle per thread (512), level 3
# stages two poses per thread.
LEVELS_BIG = [(8, 2, 4500), (4, 2, 1500), (2, 4, 700), (1, 4, 300)]


@pytest.mark.parametrize("reject", [False, True])
def test_levels_large_sets_equal_unfused_path_bitwise(torch_dev, reject):
    torch = torch_dev
    s, p, cam, poses, img = _setup(73, 5000)
    c = ctx(s, p, "bf16")
    img_d = _dev(img, torch)
    kw = dict(motion=MOTION, sigma_t=0.02, sigma_r=0.01, seed=9, iter=5)
    r = _run_levels(c, img_d, cam, LEVELS_BIG, _dev(poses, torch), torch, reject=reject, **kw)
    assert r["flags"] == 0
    u = ctx(s, p, "bf16")
    X = poses
    for L, (inv_R, B, n_out) in enumerate(LEVELS_BIG):
        g = r["levels"][L]
        po, ll, w, un = u.loc_update_particles(img_d, cam, inv_R, B, _dev(X, torch), MOTION, 0.02, 0.01, 9, 5 + L)
        rgb, op, F, E = u.loc_ray_outputs()
        assert _same(g["pose"], po.cpu().numpy()), L
        for name, ref in (("C", rgb), ("A", op), ("F", F), ("E", E), ("uncert", un)):
            assert _same(g[name], ref.cpu().numpy()), (L, name)
        if not reject:
            assert _same(g["loglik"], ll.cpu().numpy()), L
            assert _same(g["weight"], w.cpu().numpy()), L
        # the draw and the read-out from the level's own weights (after the
        # rejection when it is on), through the per-step kernels
        wl = _dev(g["weight"], torch)
        idx = u.loc_resample(wl, n_out, 9, 5 + L)
        assert _same(g["idx"], idx.cpu().numpy()), L
        if L + 1 == len(LEVELS_BIG):
            est = u.loc_pose_estimate(po, wl)
            assert _same(r["est"], est.cpu().numpy())
        X = po.cpu().numpy()[idx.cpu().numpy()]
    assert _same(r["pose"], X)


def test_levels_match_oracle_lockstep(torch_dev):
    torch = torch_dev
    s, p, cam, poses, img = _setup(72, 100)
    c = ctx(s, p, "bf16")
    kw = dict(motion=MOTION, sigma_t=0.02, sigma_r=0.01, seed=8, iter=1)
    r = _run_levels(c, _dev(img, torch), cam, LEVELS_SMALL, _dev(poses, torch), torch, reject=True, **kw)
    X = poses
    n_near = 0
    for L, (inv_R, B, n_out) in enumerate(LEVELS_SMALL):
        g = r["levels"][L]
        o = mcl.update_particles(s, p, img, cam, inv_R, B, X, MOTION, 0.02, 0.01, 8, 1 + L)
        assert np.allclose(g["pose"].reshape(-1, 12), o["pose"].reshape(-1, 12), atol=1e-12, rtol=0)
        rC = stats("C", g["C"], o["C"])
        rF = stats("F", g["F"], o["F"])
        assert rC["p99"] <= 1e-2 and rC["max"] <= 5e-2
        assert rF["p50"] <= 2e-3
        # rejection: the oracle's decisions on its own mean F, except within
        # the BF16 error of the threshold
        ll_o, rej_o = mcl.reject_1sigma(o["uncert"], o["loglik"])
        rej_g = ~np.isfinite(g["loglik"])
        U = o["uncert"]
        thr = U.mean() + U.std()
        near = np.abs(U - thr) <= 5e-3 * max(1.0, abs(thr))
        n_near += int(near.sum())
        assert np.array_equal(rej_g[~near], rej_o[~near]), L
        # l within the bound propagated from the per-ray errors (as the BF16 tests)
        keep = ~rej_g & ~rej_o
        EFg = g["E"].astype(np.float64) * g["F"]
        EFo = o["E"] * o["F"]
        bound = 4 * np.abs(EFg - EFo).sum(1) / np.minimum(EFg.sum(1), EFo.sum(1)) + 1e-3
        assert np.all(np.abs(g["loglik"][keep] - ll_o[keep]) <= bound[keep])
        # GPU rejection is its own threshold rule on its mean F
        Ug = g["uncert"].astype(np.float64)
        thr_g = Ug.mean() + Ug.std()
        assert np.array_equal(rej_g[np.abs(Ug - thr_g) > 1e-5], (Ug > thr_g)[np.abs(Ug - thr_g) > 1e-5])
        # normalisation and the draw are exact given the weights
        w_ref = mcl.normalise(g["loglik"])
        assert np.allclose(g["weight"], w_ref, atol=1e-15, rtol=1e-13)
        assert list(g["idx"]) == mcl.resample(g["weight"], n_out, 8, 1 + L)
        assert not rej_g[g["idx"]].any()
        X = g["pose"][g["idx"]]
    print("particles within the BF16 error of the rejection threshold: %d" % n_near)
    assert np.isfinite(r["pose"]).all() and np.isfinite(r["est"]).all()


@pytest.mark.parametrize("ntl,waves,blocks", [(2, 2, 7), (2, 4, 300), (2, 8, 1), (2, 8, 64), (2, 2, 2048)])
def test_levels_tile_configurations_bitwise(torch_dev, ntl, waves, blocks):
    torch = torch_dev
    s, p, cam, poses, img = _setup(73, 80)
    img_d, pose_d = _dev(img, torch), _dev(poses, torch)
    kw = dict(motion=MOTION, sigma_t=0.01, sigma_r=0.02, seed=4, iter=0, reject=True)
    base = _run_levels(ctx(s, p, "bf16"), img_d, cam, LEVELS_SMALL, pose_d, torch, **kw)
    c = ctx(s, p, "bf16")
    for L in range(len(LEVELS_SMALL)):
        c.loc_set_level_tiles(L, ntl, waves, blocks)
    r = _run_levels(c, img_d, cam, LEVELS_SMALL, pose_d, torch, **kw)
    assert _same(r["pose"], base["pose"]) and _same(r["est"], base["est"])
    for a, b in zip(r["levels"], base["levels"]):
        for k in a:
            assert _same(a[k], b[k]), k


def test_levels_autotune_and_cache(torch_dev, tmp_path):
    torch = torch_dev
    s, p, cam, poses, img = _setup(74, 200)
    img_d, pose_d = _dev(img, torch), _dev(poses, torch)
    levels = [(4, 16, 120), (2, 32, 40), (1, 64, 20)]
    cache = str(tmp_path / "tiles.jsonl")
    c = ctx(s, p, "bf16")
    chosen = c.loc_autotune_levels(img_d, cam, levels, pose_d, reps=3, cache_path=cache)
    print("chosen tiles per level:", chosen)
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 3 and all('"key": "gfx950/small-bf16-32/' in ln for ln in lines)
    c2 = ctx(s, p, "bf16")
    assert c2.loc_autotune_levels(img_d, cam, levels, pose_d, reps=3, cache_path=cache) == chosen
    assert len(open(cache).read().strip().splitlines()) == 3   # read, not re-timed
    kw = dict(sigma_t=0.01, sigma_r=0.01, seed=2, iter=9, reject=True)
    a = _run_levels(c, img_d, cam, levels, pose_d, torch, **kw)
    b = _run_levels(ctx(s, p, "bf16"), img_d, cam, levels, pose_d, torch, **kw)
    assert _same(a["pose"], b["pose"]) and _same(a["est"], b["est"])


def test_levels_graph_replays_equal_eager(torch_dev):
    torch = torch_dev
    s, p, cam, poses, img = _setup(75, 150)
    img_d, pose_d = _dev(img, torch), _dev(poses, torch)
    levels = [(4, 16, 90), (2, 32, 40), (1, 48, 16)]
    g = ctx(s, p, "bf16")
    g.loc_set_graph_mode(True)
    e = ctx(s, p, "bf16")
    po = torch.empty((16, 3, 4), dtype=torch.float64, device="cuda")
    est = torch.empty((3, 4), dtype=torch.float64, device="cuda")
    for rep, (seed, it, st, sr) in enumerate([(1, 0, 0.02, 0.01), (1, 3, 0.0, 0.0), (9, 7, 0.05, 0.03), (2, 2, 0.01, 0.0)]):
        mo = MOTION if rep % 2 else None
        g.loc_update_levels(img_d, cam, levels, pose_d, motion=mo, sigma_t=st, sigma_r=sr, seed=seed, iter=it,
                            reject=True, pose_out=po, est_out=est)
        torch.cuda.synchronize()
        got = (po.cpu().numpy(), est.cpu().numpy(),
               [{k: v.cpu().numpy() for k, v in g.loc_level_outputs(L).items()} for L in range(3)])
        # eager work between replays
        ref = _run_levels(e, img_d, cam, levels, pose_d, torch, motion=mo, sigma_t=st, sigma_r=sr, seed=seed,
                          iter=it, reject=True)
        assert _same(got[0], ref["pose"]) and _same(got[1], ref["est"]), rep
        for L in range(3):
            for k in got[2][L]:
                assert _same(got[2][L][k], ref["levels"][L][k]), (rep, L, k)
        assert g.loc_sync() == 0


def test_levels_full_c2f_workload(torch_dev):
    """800x800 image, levels 1/4, 1/2, 1 with 16, 64, 256 rays per particle,
    1000 -> 300 -> 100 particles, 1-sigma rejection, graph replay: weights
    normalise at every level, rejected particles are never drawn, and three
    sampled particles per level match the oracle's log-likelihood."""
    torch = torch_dev
    s, p, cam, poses, img = _setup(76, 1000)
    levels = [(4, 16, 300), (2, 64, 100), (1, 256, 100)]
    c = ctx(s, p, "bf16")
    c.loc_set_graph_mode(True)
    kw = dict(sigma_t=0.02, sigma_r=math.radians(1.0), seed=11, iter=0, reject=True)
    r = _run_levels(c, _dev(img, torch), cam, levels, _dev(poses, torch), torch, **kw)
    assert r["flags"] == 0
    X = poses
    for L, (inv_R, B, n_out) in enumerate(levels):
        g = r["levels"][L]
        assert abs(g["weight"].sum() - 1.0) <= 1e-12
        rej = ~np.isfinite(g["loglik"])
        print("level %d: %d particles, %d rejected" % (L, g["weight"].size, rej.sum()))
        assert 0 < rej.sum() < g["weight"].size // 2
        assert not rej[g["idx"]].any()
        sub = [0, len(X) // 2, len(X) - 1]
        o = mcl.update_particles(s, p, img, cam, inv_R, B, X, None, kw["sigma_t"], kw["sigma_r"], 11, L, subset=sub)
        assert np.allclose(g["pose"][sub].reshape(3, 12), o["pose"].reshape(3, 12), atol=1e-12, rtol=0)
        EFg = g["E"][sub].astype(np.float64) * g["F"][sub]
        EFo = o["E"] * o["F"]
        raw = 4 * (math.log(B) - np.log(np.maximum(EFg.sum(1), 1e-12)))
        stats("loglik L%d" % L, raw, o["loglik"])
        bound = 4 * np.abs(EFg - EFo).sum(1) / np.minimum(EFg.sum(1), EFo.sum(1)) + 1e-3
        assert np.all(np.abs(raw - o["loglik"]) <= bound)
        rC = stats("C L%d" % L, g["C"][sub], o["C"])
        assert rC["p99"] <= 1e-2
        X = g["pose"][g["idx"]]
    assert np.isfinite(r["est"]).all()
