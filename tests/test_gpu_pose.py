"""GPU parity of the pose gather after resampling and the pose read-out
against the FP64 oracle, and a short localisation loop (predict, weight,
resample, gather, read-out) against the oracle's loop on the same seeds.

Bars: gather bit-exact; read-out within 1e-10 of the oracle's SVD form
(both FP64); loop estimate within 1 cm and 0.5 degree of the oracle's."""
import numpy as np
import pytest

from oracle import mcl, se3
from paper_2406_12202_amd import synth
from parity_util import ctx, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def small_ctx():
    s, p, _, _, _ = inputs("small", 51)
    return ctx(s, p)


def _dev(x, torch):
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def _haar_set(seed, n, spread_deg):
    """n poses around a random rotation, rotations perturbed by about spread_deg."""
    rng = np.random.default_rng(seed)
    R0 = synth.haar_rotation(rng)
    out = np.zeros((n, 3, 4))
    for i in range(n):
        phi = rng.standard_normal(3) * np.deg2rad(spread_deg)
        E = se3.exp_se3(np.zeros(3), phi)
        out[i, :, :3] = R0 @ E[:, :3]
        out[i, :, 3] = rng.uniform(-2, 2, 3)
    return out


@pytest.mark.parametrize("n_in,n_out", [(1, 1), (7, 300), (1000, 1000), (4096, 777)])
def test_gather_bit_exact(torch_dev, small_ctx, n_in, n_out):
    torch = torch_dev
    rng = np.random.default_rng(n_in + n_out)
    poses = rng.standard_normal((n_in, 3, 4))
    idx = rng.integers(0, n_in, n_out).astype(np.int32)
    got = small_ctx.loc_gather_poses(_dev(poses, torch), _dev(idx, torch)).cpu().numpy()
    assert np.array_equal(got, poses[idx])


def test_gather_after_resample_matches_oracle(torch_dev, small_ctx):
    torch = torch_dev
    rng = np.random.default_rng(5)
    w = rng.exponential(size=2000)
    w[rng.random(2000) < 0.3] = 0.0
    w /= w.sum()
    poses = rng.standard_normal((2000, 3, 4))
    idx = small_ctx.loc_resample(_dev(w, torch), 1500, seed=8, iter=2)
    got = small_ctx.loc_gather_poses(_dev(poses, torch), idx).cpu().numpy()
    ref_idx = mcl.resample(w, 1500, 8, 2)
    assert np.array_equal(got, poses[ref_idx])


@pytest.mark.parametrize("seed,n,spread", [(1, 1, 0.0), (2, 37, 2.0), (3, 1000, 10.0), (4, 5000, 40.0),
                                           (5, 100, 120.0)])
def test_pose_estimate_matches_oracle(torch_dev, small_ctx, seed, n, spread):
    torch = torch_dev
    poses = _haar_set(seed, n, spread)
    w = np.random.default_rng(seed + 100).exponential(size=n)
    if n > 10:
        w[::7] = 0.0                     # resampled-away particles carry no weight
    est = small_ctx.loc_pose_estimate(_dev(poses, torch), _dev(w, torch)).cpu().numpy()
    ref = se3.pose_estimate(poses, w)
    d = np.abs(est - ref).max()
    print("n=%d spread=%.0f deg: max |d| %.3e" % (n, spread, d))
    assert d <= 1e-10
    assert small_ctx.loc_sync() == 0


def test_pose_estimate_reflection_case(torch_dev, small_ctx):
    """A weighted rotation sum with negative determinant takes the
    det(U V^T) = -1 branch of the chordal mean."""
    torch = torch_dev
    found = None
    for seed in range(500):
        rng = np.random.default_rng(seed)
        R = np.stack([synth.haar_rotation(rng) for _ in range(4)])
        w = rng.exponential(size=4)
        M = np.einsum("i,ijk->jk", w / w.sum(), R)
        if np.linalg.det(M) < -1e-3:
            found = (R, w)
            break
    assert found is not None
    R, w = found
    poses = np.zeros((4, 3, 4))
    poses[:, :, :3] = R
    est = small_ctx.loc_pose_estimate(_dev(poses, torch), _dev(w, torch)).cpu().numpy()
    ref = se3.pose_estimate(poses, w)
    assert abs(np.linalg.det(est[:, :3]) - 1.0) <= 1e-12
    assert np.abs(est - ref).max() <= 1e-10


def test_pose_estimate_degenerate_weights(torch_dev, small_ctx):
    torch = torch_dev
    poses = _haar_set(9, 16, 5.0)
    w = np.zeros(16)
    w[3] = -1.0
    w[4] = np.nan
    small_ctx.loc_sync()
    est = small_ctx.loc_pose_estimate(_dev(poses, torch), _dev(w, torch)).cpu().numpy()
    assert np.isnan(est).all()
    assert small_ctx.loc_sync() & 1


def test_localisation_loop_matches_oracle(torch_dev):
    """Four filter iterations on the small map: predict with motion noise,
    weight, resample, gather; read out the pose each iteration."""
    torch = torch_dev
    s, p, cam, poses, img = inputs("small", 52, N=64)
    c = ctx(s, p)
    motion = np.eye(4)[:3]
    motion[:, 3] = [0.01, 0.0, -0.005]
    st, sr = 0.02, 0.01
    g_pose = _dev(poses, torch)
    o_pose = poses.copy()
    for it in range(4):
        po, ll, w, _ = c.loc_update_particles(_dev(img, torch).float(), cam, 1, 16, g_pose, motion, st, sr,
                                              seed=13, iter=it)
        est_g = c.loc_pose_estimate(po, w).cpu().numpy()
        idx = c.loc_resample(w, 64, seed=13, iter=it)
        g_pose = c.loc_gather_poses(po, idx)
        assert c.loc_sync() == 0
        o = mcl.update_particles(s, p, img, cam, 1, 16, o_pose, motion, st, sr, 13, it)
        est_o = se3.pose_estimate(o["pose"], o["weight"])
        ridx = mcl.resample(o["weight"], 64, 13, it)
        o_pose = np.asarray(o["pose"])[ridx]
        dt, dr = se3.pose_errors(est_g, est_o)
        same = int((idx.cpu().numpy() == ridx).sum())
        print("iter %d: |dt| %.3e m  |dR| %.3e deg  same indices %d/64" % (it, dt, dr, same))
        assert dt <= 0.01 and dr <= 0.5
