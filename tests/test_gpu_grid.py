"""GPU parity of the multi-resolution grid map (Sec. IV-B map type) against the
FP64 oracle (oracle/grid.py through mcl.update_particles).

The grid path computes in float32: the cell coordinate p = u N_l carries a
relative rounding of about 2^-24 times N_l (up to 2048), so the trilinear
weights move by up to ~1.2e-4 and a level's features, which are continuous
across cell faces, by that times the spread of the corner entries (up to ~3
for N(0, 0.5^2) entries), ~4e-4; the tiny MLP's density logit takes them
with a gain of about 3, and softplus turns a logit error dz into a relative
density error of at most dz, so each sample's optical depth carries a
relative error of about 1e-3 per level: EPS_GRID = 4e-3 over 16 levels of
independent signs.  Per ray, a relative optical-depth error eps moves the
opacity A = 1 - e^-tau by (1 - A) tau eps, and the colour by as much plus
the colour head's own share of the feature error (sigmoid slope <= 1/4 on a
logit error of ~1e-3).  Bars: every ray within (1 - A) tau EPS_GRID + 1e-4
(opacity) and + 3e-4 (colour), tau = -ln(1 - A) of the oracle; colour and
opacity p99 <= 5e-4; F: 99% of rays within 2e-3 and all within 0.1
(thin-density crossings amplify rounding as for the NeRF map);
log-likelihood 1e-3; weights 1e-4 absolute (a weight moves by at most
w (1 - w) |dl| <= |dl| / 4).
"""
import numpy as np
import pytest

from oracle import mcl
from paper_2406_12202_amd import synth
from parity_util import frac_over, stats

pytestmark = pytest.mark.gpu

TOL = dict(C=5e-4, F=2e-3, F_MAX=0.1, L=1e-3, W=5e-2)
EPS_GRID = 4e-3


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _ctx(spec, params):
    from paper_2406_12202_amd import binding
    return binding.Context(spec, params)


def _run(torch, ctx, img, cam, inv_R, B, poses, seed, it, sigma_t=0.0, sigma_r=0.0):
    dev = torch.device("cuda", 0)
    po, ll, w, un = ctx.loc_update_particles(torch.as_tensor(img, device=dev), cam, inv_R, B,
                                             torch.as_tensor(poses, device=dev).contiguous(), None, sigma_t, sigma_r,
                                             seed, it)
    rgb, op, F, E = ctx.loc_ray_outputs()
    return dict(pose=po.cpu().numpy(), loglik=ll.cpu().numpy(), weight=w.cpu().numpy(), C=rgb.cpu().numpy(),
                A=op.cpu().numpy(), F=F.cpu().numpy(), flags=ctx.loc_sync())


def _compare(g, o, idx):
    assert np.allclose(g["pose"][idx].reshape(len(idx), 12), o["pose"].reshape(len(idx), 12), atol=1e-12, rtol=0)
    rC = stats("C", g["C"][idx], o["C"])
    rA = stats("A", g["A"][idx], o["A"])
    rF = stats("F", g["F"][idx], o["F"])
    rL = stats("loglik", g["loglik"][idx], o["loglik"])
    assert rC["p99"] <= TOL["C"] and rA["p99"] <= TOL["C"]
    Ao = np.clip(o["A"], 0.0, 1.0 - 1e-12)
    tau_term = (1.0 - Ao) * -np.log1p(-Ao) * EPS_GRID
    okA = np.abs(g["A"][idx] - o["A"]) <= tau_term + 1e-4
    okC = np.all(np.abs(g["C"][idx] - o["C"]) <= tau_term[..., None] + 3e-4, axis=-1)
    print("rays within the per-ray bound: opacity %.4f, colour %.4f of %d" % (okA.mean(), okC.mean(), okA.size))
    assert okA.all() and okC.all()
    ll = g["loglik"][idx]
    ws = np.exp(ll - ll.max())
    dw = np.abs(ws / ws.sum() - o["weight"]).max()
    print("weight     max=%.3e" % dw)
    assert dw <= 1e-4
    assert frac_over(g["F"][idx], o["F"], TOL["F"]) <= 0.01
    assert rF["max"] <= TOL["F_MAX"]
    assert rL["max"] <= TOL["L"]


def test_grid_map_update_full_size_sampled_particles(torch_dev):
    """16 levels of 2^19 entries, 400 particles x 64 rays x (64 + 128
    hierarchical) samples; three particles checked against the oracle."""
    torch = torch_dev
    spec = synth.grid_spec()
    params = synth.grid_params(spec, 1)
    cam = synth.camera("nerf")
    poses = synth.particles("nerf", 1)
    img = synth.observation("nerf", 1)
    ctx = _ctx(spec, params)
    g = _run(torch, ctx, img, cam, 1, 64, poses, 5, 2, sigma_t=0.01, sigma_r=0.01)
    idx = [0, 137, 399]
    o = mcl.update_particles(spec, params, img, cam, 1, 64, poses, None, 0.01, 0.01, 5, 2, subset=idx)
    _compare(g, o, idx)
    assert np.all(np.isfinite(g["loglik"])) and abs(g["weight"].sum() - 1.0) < 1e-12
    ctx.close()


def test_grid_map_chunk_boundary_inside_a_ray(torch_dev):
    """400 particles x 64 rays x (64 + 112) samples: the fine set of 2,867,200
    samples is evaluated in two chunks of at most 2^21, and the boundary,
    sample 2,097,152, falls inside ray 18724 (particle 292, ray 36, fine
    sample 64 of 112; a ray through the box); that particle, the first and
    the last against the oracle."""
    torch = torch_dev
    spec = synth.grid_spec(n_coarse=64, n_fine=112)
    params = synth.grid_params(spec, 8)
    cam = synth.camera("nerf")
    poses = synth.particles("nerf", 8)
    img = synth.observation("nerf", 8)
    ctx = _ctx(spec, params)
    g = _run(torch, ctx, img, cam, 1, 64, poses, 9, 1)
    assert (1 << 21) // 112 == 18724 and (1 << 21) % 112 == 64
    idx = [0, 292, 399]
    o = mcl.update_particles(spec, params, img, cam, 1, 64, poses, None, 0.0, 0.0, 9, 1, subset=idx)
    assert o["A"][1][36] > 0.1      # the boundary ray is not empty
    _compare(g, o, idx)
    ctx.close()


@pytest.mark.parametrize("levels,L_dir,log2_table", [(4, 4, 10), (8, 2, 12)])
def test_grid_map_small_tables_dense_hash_and_box_edge(torch_dev, levels, L_dir, log2_table):
    """Small tables (dense coarse levels, hashed fine ones, many collisions)
    and a box of half-size 3 that the rays leave, so samples outside it are
    empty; all particles checked."""
    torch = torch_dev
    spec = synth.grid_spec(n_coarse=32, n_fine=0, levels=levels, L_dir=L_dir, log2_table=log2_table, n_min=4,
                           n_max=96, bound=3.0)
    params = synth.grid_params(spec, 2)
    cam = synth.camera("small")
    poses = synth.particles("small", 2, N=12)
    img = synth.observation("small", 2)
    ctx = _ctx(spec, params)
    g = _run(torch, ctx, img, cam, 2, 16, poses, 7, 1)
    o = mcl.update_particles(spec, params, img, cam, 2, 16, poses, None, 0.0, 0.0, 7, 1)
    _compare(g, o, list(range(12)))
    assert np.all(g["A"] >= 0.0) and np.all(g["A"] <= 1.0)
    ctx.close()


def test_grid_map_render_image_sampled(torch_dev):
    torch = torch_dev
    spec = synth.grid_spec(n_coarse=64, n_fine=64)
    params = synth.grid_params(spec, 3)
    cam = synth.camera("nerf")
    pose = synth.gt_pose("nerf", 3)
    dev = torch.device("cuda", 0)
    ctx = _ctx(spec, params)
    rgb = ctx.loc_render_image(cam, 4, torch.as_tensor(pose, device=dev).contiguous(), seed=2, iter=0)
    rgb = rgb.cpu().numpy().astype(np.float64)
    Wl = cam[0] // 4
    rng = np.random.default_rng(3)
    pix = sorted(set(rng.choice(Wl * (cam[1] // 4), 40, replace=False).tolist()))
    W, H, fx, fy, cx, cy = cam
    rays = mcl.particle_rays(pose, pix, Wl, (fx / 4, fy / 4, cx / 4, cy / 4))
    r = mcl.render_rays(spec, mcl.unpack_map(spec, params), rays, [(0, p) for p in pix], 2, 0)
    rc = stats("C", rgb.reshape(-1, 3)[pix], r["C"])
    assert rc["max"] <= TOL["C"]
    ctx.close()


def test_grid_map_rejects_unsupported(torch_dev):
    from paper_2406_12202_amd.binding import LocError
    spec = synth.grid_spec(levels=5)
    with pytest.raises(LocError):
        _ctx(spec, synth.grid_params(spec, 4))
    spec = synth.grid_spec(L_dir=3)
    with pytest.raises(LocError):
        _ctx(spec, synth.grid_params(spec, 4))


def test_grid_map_with_proposal_placement(torch_dev):
    """Proposal-placed fine samples (a seeded, untrained proposal network) on
    the grid map; all particles of a small workload checked."""
    torch = torch_dev
    spec = synth.grid_spec(n_coarse=32, n_fine=16, levels=8, log2_table=14, n_min=8, n_max=256)
    params = synth.grid_params(spec, 5)
    prop = synth.proposal_params(5)
    cam = synth.camera("small")
    poses = synth.particles("small", 5, N=6)
    img = synth.observation("small", 5)
    ctx = _ctx(spec, params)
    ctx.loc_set_proposal(prop)
    ctx.loc_set_fine_mode(1)
    g = _run(torch, ctx, img, cam, 1, 12, poses, 3, 4)
    o = mcl.update_particles(spec, params, img, cam, 1, 12, poses, None, 0.0, 0.0, 3, 4, proposal=prop)
    _compare(g, o, list(range(6)))
    ctx.close()


def test_grid_map_in_the_localisation_loop(torch_dev):
    """Two iterations of the localisation loop on a small grid map: the loop's
    trace against oracle updates of the same sets (weights), indices exact."""
    torch = torch_dev
    spec = synth.grid_spec(n_coarse=24, n_fine=0, levels=4, log2_table=12, n_min=4, n_max=64, L_dir=4)
    params = synth.grid_params(spec, 6)
    cam = synth.camera("small")
    poses = synth.particles("small", 6, N=10)
    img = synth.observation("small", 6)
    dev = torch.device("cuda", 0)
    ctx = _ctx(spec, params)
    stages = [(2, 8, 10, 1e9), (1, 8, 8, 0.0)]
    out = ctx.loc_localize(torch.as_tensor(img, device=dev), cam, stages, 2,
                           torch.as_tensor(poses, device=dev).contiguous(), seed=7, trace_capacity=20)
    tw = out["trace"]["weight"].cpu().numpy()
    tp = out["trace"]["pose"].cpu().numpy()
    ti = out["trace"]["idx"].cpu().numpy()
    assert [r["stage"] for r in out["steps"]] == [0, 1]
    o0 = mcl.update_particles(spec, params, img, cam, 2, 8, poses, None, 0.0, 0.0, 7, 0)
    big = o0["weight"] > 1e-6
    assert np.all(np.abs(tw[:10] - o0["weight"])[big] <= TOL["W"] * o0["weight"][big])
    idx0 = mcl.resample(tw[:10], 8, 7, 0)
    assert np.array_equal(ti[:8], np.asarray(idx0, np.int32))
    X1 = tp[:10][np.asarray(idx0)]
    o1 = mcl.update_particles(spec, params, img, cam, 1, 8, X1, None, 0.0, 0.0, 7, 1)
    big = o1["weight"] > 1e-6
    assert np.all(np.abs(tw[10:18] - o1["weight"])[big] <= TOL["W"] * o1["weight"][big])
    ctx.close()


def test_grid_map_level_path_is_unsupported(torch_dev):
    torch = torch_dev
    from paper_2406_12202_amd.binding import LocError
    spec = synth.grid_spec(n_coarse=32, n_fine=0, levels=4, log2_table=12, n_min=4, n_max=64)
    ctx = _ctx(spec, synth.grid_params(spec, 7))
    dev = torch.device("cuda", 0)
    cam = synth.camera("small")
    with pytest.raises(LocError):
        ctx.loc_update_levels(torch.as_tensor(synth.observation("small", 7), device=dev), cam, [(1, 4, 4)],
                              torch.as_tensor(synth.particles("small", 7, N=4), device=dev).contiguous())
    ctx.close()
