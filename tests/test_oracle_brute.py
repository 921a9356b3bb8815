"""Brute-force pins of the FP64 oracle's whole weighting pass and of its two
least constrained steps.

1. An independent 50-digit evaluator (mpmath) of one weighting pass of
   Alg. 1 -- prediction by the SE(3) exponential of a Gaussian twist, the
   downscaled observation, pixel rays, stratified coarse samples, the map
   F(x, d) -> (c, sigma) with its positional encoding, hierarchical or
   proposal-guided fine samples, the Eq. 1 quadrature, the Eq. 5 quantiles,
   the Eq. 6 score and the Eq. 3 normalisation -- on a tiny random map that is
   far from constant, so that where the fine samples land changes every
   output.  It shares no code with the oracle: only the Philox words (the
   generator's published definition, pinned by its known-answer vectors) and
   the documented flat parameter order are common.  The oracle must agree
   with it to 1e-12.
2. Hierarchical placement on a two-slab density in closed form: the coarse
   weights telescope to differences of exponentials of the sample depths, so
   the normalised cumulative pdf mass (weights plus 1e-5 per unit length) and
   the inverse-CDF fine depths are known exactly.
3. The chordal-mean rotation of the pose read-out against Davenport's
   q-method on a constructed set whose weighted rotation sum has negative
   determinant (the branch where the SVD form needs its det(U V^T) sign).
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import mcl, philox as px, proposal as pr, render as rd, se3
from paper_2406_12202_amd import synth

DPS = 50


# ----------------------------------------------------------------------------- generator words

def _words(seed, it, stream, c0, c1, group):
    return [int(w) for w in px.draw_words(seed, it, stream, c0, c1, group)]


def _word(seed, it, stream, c0, c1, index):
    return _words(seed, it, stream, c0, c1, index // 4)[index % 4]


def _u24(w):
    return mp.mpf(w >> 8) / 2 ** 24


def _uopen(w):
    return (mp.mpf(w) + mp.mpf(1) / 2) / 2 ** 32


# ----------------------------------------------------------------------------- 50-digit evaluator

class MpMap:
    """F(x, d) -> (sigma, rgb) from the documented flat parameter order:
    hidden layers (W row-major, then b), with [h, gamma(x)] entering the skip
    layer; density head; then feature, direction and colour layers, or a
    colour layer on [h, gamma(d)] when there is no direction layer."""

    def __init__(self, spec, flat):
        self.s = spec
        vals = [mp.mpf(float(v)) for v in np.asarray(flat, dtype=np.float32)]
        D, Wd, skip = spec["n_layers"], spec["width"], spec["skip_layer"]
        nx, nd = 3 + 6 * spec["L_xyz"], 3 + 6 * spec["L_dir"]
        shapes = []
        for l in range(D):
            shapes.append((Wd, nx if l == 0 else (Wd + nx if l == skip else Wd)))
        shapes.append((1, Wd))
        if spec["dir_width"] > 0:
            shapes += [(Wd, Wd), (spec["dir_width"], Wd + nd), (3, spec["dir_width"])]
        else:
            shapes.append((3, Wd + nd))
        self.layers, pos = [], 0
        for o, i in shapes:
            W = [vals[pos + r * i: pos + (r + 1) * i] for r in range(o)]
            pos += o * i
            b = vals[pos: pos + o]
            pos += o
            self.layers.append((W, b))
        assert pos == len(vals)

    @staticmethod
    def enc(p, L):
        out = list(p)
        for l in range(L):
            out += [mp.sin(2 ** l * mp.pi * c) for c in p]
            out += [mp.cos(2 ** l * mp.pi * c) for c in p]
        return out

    @staticmethod
    def lin(Wb, u):
        W, b = Wb
        return [sum((w * x for w, x in zip(row, u)), mp.mpf(0)) + bb for row, bb in zip(W, b)]

    def __call__(self, x, d):
        s = self.s
        D = s["n_layers"]
        gx, gd = self.enc(x, s["L_xyz"]), self.enc(d, s["L_dir"])
        h = gx
        for l in range(D):
            if l == s["skip_layer"] and l > 0:
                h = h + gx
            h = [max(v, 0) for v in self.lin(self.layers[l], h)]
        z = self.lin(self.layers[D], h)[0]
        sigma = mp.log1p(mp.exp(z))
        if s["dir_width"] > 0:
            f = self.lin(self.layers[D + 1], h)
            g = [max(v, 0) for v in self.lin(self.layers[D + 2], f + gd)]
            zc = self.lin(self.layers[D + 3], g)
        else:
            zc = self.lin(self.layers[D + 1], h + gd)
        return sigma, [1 / (1 + mp.exp(-v)) for v in zc]


def _mp_exp_twist(rho, phi):
    """Exp of the 4x4 twist matrix by mpmath's own matrix exponential."""
    M = mp.zeros(4, 4)
    M[0, 1], M[0, 2], M[1, 2] = -phi[2], phi[1], -phi[0]
    M[1, 0], M[2, 0], M[2, 1] = phi[2], -phi[1], phi[0]
    for r in range(3):
        M[r, 3] = rho[r]
    return mp.expm(M)


def _mp_predict(pose, i, seed, it, st, sr):
    w = _words(seed, it, px.S_MOTION, i, 0, 0) + _words(seed, it, px.S_MOTION, i, 0, 1)
    u = [_uopen(x) for x in w]
    g = []
    for a in range(3):
        r = mp.sqrt(-2 * mp.log(u[2 * a]))
        g += [r * mp.cos(2 * mp.pi * u[2 * a + 1]), r * mp.sin(2 * mp.pi * u[2 * a + 1])]
    E = _mp_exp_twist([st * v for v in g[:3]], [sr * v for v in g[3:]])
    X = mp.matrix(4, 4)
    for r in range(3):
        for c in range(4):
            X[r, c] = mp.mpf(float(pose[r, c]))
    X[3, 3] = 1
    return X * E


def _composite(t, sig, rgb, far):
    S = len(t)
    dl = [t[k + 1] - t[k] for k in range(S - 1)] + [far - t[-1]]
    logT = [mp.mpf(0)]
    for k in range(S):
        logT.append(logT[-1] - sig[k] * dl[k])
    w = [mp.exp(logT[k]) * (1 - mp.exp(-sig[k] * dl[k])) for k in range(S)]
    C = [sum((w[k] * rgb[k][c] for k in range(S)), mp.mpf(0)) for c in range(3)]
    return w, logT, C, sum(w, mp.mpf(0)), dl


def _crossing(t, sig, logT, level, strict):
    lv = mp.log(level)
    for k in range(len(t)):
        if (logT[k + 1] < lv) if strict else (logT[k + 1] <= lv):
            return t[k] + (logT[k] - lv) / sig[k]
    return None


def _inverse_cdf(starts, widths, mass, u):
    tot = sum(mass, mp.mpf(0))
    c = [mp.mpf(0)]
    for m in mass:
        c.append(c[-1] + m / tot)
    k = max(b for b in range(len(mass)) if c[b] <= u)
    return starts[k] + (u - c[k]) / (c[k + 1] - c[k]) * widths[k]


def _mp_proposal_hist(theta, o, d):
    v = [mp.mpf(float(x)) for x in np.asarray(theta, dtype=np.float32)]
    x = MpMap.enc(o, 6) + MpMap.enc(d, 6)
    pos = 0
    for n_out, n_in, relu in ((64, 78, True), (64, 64, True), (32, 64, False)):
        W = [v[pos + r * n_in: pos + (r + 1) * n_in] for r in range(n_out)]
        pos += n_out * n_in
        b = v[pos: pos + n_out]
        pos += n_out
        y = MpMap.lin((W, b), x)
        x = [max(q, 0) for q in y] if relu else y
    m = max(x)
    e = [mp.exp(q - m) for q in x]
    return [q / sum(e) for q in e]


def mp_update(spec, flat, image, cam, inv_R, B, poses, st, sr, seed, it, proposal=None):
    """One weighting pass of Alg. 1 at 50 digits; returns per-particle C, A,
    F (B values each), the log-likelihoods and the normalised weights."""
    with mp.workdps(DPS):
        F_map = MpMap(spec, flat)
        near, far = mp.mpf(spec["near"]), mp.mpf(spec["far"])
        alpha, tau = mp.mpf(spec["alpha"]), mp.mpf(spec["tau"])
        Sc, Sf = spec["n_coarse"], spec["n_fine"]
        W, H, fx, fy, cx, cy = cam
        s = int(inv_R)
        Wl, Hl = W // s, H // s
        img = np.asarray(image, dtype=np.float32)
        pix = [(_word(seed, it, px.S_PIX, j, 0, 0) * (Wl * Hl)) >> 32 for j in range(B)]
        obs = []
        for p in pix:
            u, v = p % Wl, p // Wl
            blk = [[mp.mpf(float(img[v * s + a, u * s + b, c])) for a in range(s) for b in range(s)]
                   for c in range(3)]
            obs.append([sum(q, mp.mpf(0)) / (s * s) for q in blk])
        kx, ky = mp.mpf(fx) / s, mp.mpf(fy) / s
        ox, oy = mp.mpf(cx) / s, mp.mpf(cy) / s
        out = dict(C=[], A=[], F=[], loglik=[])
        for i in range(poses.shape[0]):
            X = _mp_predict(poses[i], i, seed, it, mp.mpf(st), mp.mpf(sr))
            Ssum = mp.mpf(0)
            Ci, Ai, Fi = [], [], []
            for j, p in enumerate(pix):
                u, v = p % Wl, p // Wl
                dc = [(u + mp.mpf(1) / 2 - ox) / kx, -(v + mp.mpf(1) / 2 - oy) / ky, mp.mpf(-1)]
                dw = [sum(X[r, c] * dc[c] for c in range(3)) for r in range(3)]
                nrm = mp.sqrt(sum(q * q for q in dw))
                d = [q / nrm for q in dw]
                o = [X[r, 3] for r in range(3)]
                dt = (far - near) / Sc
                tc = [near + (k + (_u24(_word(seed, it, px.S_JIT_COARSE, i, j, k)) if spec["jitter"] else 0)) * dt
                      for k in range(Sc)]
                ev = [F_map([o[c] + t * d[c] for c in range(3)], d) for t in tc]
                samples = [(t, 0, e) for t, e in zip(tc, ev)]
                if Sf > 0:
                    um = [(m + (_u24(_word(seed, it, px.S_JIT_FINE, i, j, m)) if spec["jitter"] else mp.mpf(1) / 2))
                          / Sf for m in range(Sf)]
                    if proposal is None:
                        w, _, _, _, dl = _composite(tc, [e[0] for e in ev], [e[1] for e in ev], far)
                        mass = [w[k] + mp.mpf("1e-5") * dl[k] for k in range(Sc)]
                        tf = [_inverse_cdf(tc, dl, mass, q) for q in um]
                    else:
                        ph = _mp_proposal_hist(proposal, o, d)
                        bw = (far - near) / 32
                        mass = [mp.mpf("0.99") * q + mp.mpf("0.01") / 32 for q in ph]
                        tf = [_inverse_cdf([near + b * bw for b in range(32)], [bw] * 32, mass, q) for q in um]
                    samples += [(t, 1, F_map([o[c] + t * d[c] for c in range(3)], d)) for t in tf]
                samples.sort(key=lambda e: (e[0], e[1]))
                t = [e[0] for e in samples]
                sig = [e[2][0] for e in samples]
                w, logT, C, A, _ = _composite(t, sig, [e[2][1] for e in samples], far)
                zt = _crossing(t, sig, logT, 1 - alpha, strict=False)
                zo = _crossing(t, sig, logT, alpha, strict=True)
                zo = far if zo is None else zo
                Fj = tau if zt is None else max(zo - zt, tau)
                E = sum(((obs[j][c] - C[c]) ** 2 for c in range(3)), mp.mpf(0))
                Ssum += E * Fj
                Ci.append([float(c) for c in C])
                Ai.append(float(A))
                Fi.append(float(Fj))
            out["C"].append(Ci)
            out["A"].append(Ai)
            out["F"].append(Fi)
            out["loglik"].append(4 * (mp.log(B) - mp.log(max(Ssum, mp.mpf("1e-12")))))
        m = max(out["loglik"])
        e = [mp.exp(q - m) for q in out["loglik"]]
        out["weight"] = [float(q / sum(e)) for q in e]
        out["loglik"] = [float(q) for q in out["loglik"]]
        for k in ("C", "A", "F"):
            out[k] = np.array(out[k])
        return out


# ----------------------------------------------------------------------------- tiny scenes

TINY = dict(n_layers=2, width=4, skip_layer=1, L_xyz=2, L_dir=1, dir_width=4,
            near=2.0, far=6.0, alpha=0.05, tau=0.1, jitter=1, n_coarse=4, n_fine=4)


def _tiny_map(spec, seed):
    """Random weights of order one with a density head that swings the
    density between near-empty and opaque within the sampled span."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, o, i in rd.layer_shapes(spec):
        W = rng.standard_normal((o, i)) * (1.5 / math.sqrt(i))
        b = 0.3 * rng.standard_normal(o)
        if (o, i) == (1, spec["width"]):
            W *= 3.0
            b[:] = -1.0
        parts += [W.ravel(), b]
    return np.concatenate(parts).astype(np.float32)


def _tiny_scene(seed, spec):
    rng = np.random.default_rng(seed + 100)
    cam = (8, 8, 6.0, 6.0, 4.0, 4.0)
    poses = np.stack([synth.lookat(4.0 * v / np.linalg.norm(v), target=0.3 * rng.standard_normal(3))
                      for v in rng.standard_normal((2, 3))])
    img = rng.random((8, 8, 3)).astype(np.float32)
    return _tiny_map(spec, seed), cam, poses, img


def _compare(o, m):
    assert np.allclose(o["C"], m["C"], rtol=0, atol=1e-12)
    assert np.allclose(o["A"], m["A"], rtol=0, atol=1e-12)
    assert np.allclose(o["F"], m["F"], rtol=0, atol=1e-11)
    assert np.allclose(o["loglik"], m["loglik"], rtol=0, atol=1e-10)
    assert np.allclose(o["weight"], m["weight"], rtol=0, atol=1e-12)


@pytest.mark.parametrize("dir_width", [4, 0])
@pytest.mark.parametrize("seed", [1, 2])
def test_whole_pass_hierarchical_against_50_digit_evaluator(seed, dir_width):
    spec = dict(TINY, dir_width=dir_width, skip_layer=1 if dir_width else -1)
    p, cam, poses, img = _tiny_scene(seed, spec)
    kw = dict(seed=40 + seed, it=3)
    o = mcl.update_particles(spec, p, img, cam, 2, 2, poses, None, 0.05, 0.03, **kw)
    m = mp_update(spec, p, img, cam, 2, 2, poses, 0.05, 0.03, **kw)
    # the scene is informative: opacities away from 0 and 1, fine samples
    # placed where the coarse weights put them
    assert np.any((m["A"] > 0.05) & (m["A"] < 0.95))
    _compare(o, m)


@pytest.mark.parametrize("seed", [3, 4])
def test_whole_pass_proposal_against_50_digit_evaluator(seed):
    spec = dict(TINY)
    p, cam, poses, img = _tiny_scene(seed, spec)
    theta = synth.proposal_params(seed)
    kw = dict(seed=50 + seed, it=1)
    o = mcl.update_particles(spec, p, img, cam, 1, 2, poses, None, 0.02, 0.01, proposal=theta, **kw)
    m = mp_update(spec, p, img, cam, 1, 2, poses, 0.02, 0.01, proposal=theta, **kw)
    assert np.any((m["A"] > 0.05) & (m["A"] < 0.95))
    _compare(o, m)


def test_whole_pass_without_jitter_against_50_digit_evaluator():
    spec = dict(TINY, jitter=0, n_coarse=5, n_fine=3)
    p, cam, poses, img = _tiny_scene(7, spec)
    o = mcl.update_particles(spec, p, img, cam, 2, 3, poses, None, 0.0, 0.0, seed=9, it=0)
    m = mp_update(spec, p, img, cam, 2, 3, poses, 0.0, 0.0, seed=9, it=0)
    _compare(o, m)


# ----------------------------------------------------------------------------- two-slab placement

@pytest.mark.parametrize("jitter", [0, 1])
def test_hierarchical_placement_on_two_slabs_in_closed_form(jitter, monkeypatch):
    """Density 0 before the plane z = -a and s behind it, seen along -z from
    z = 4: a sample at depth t_k >= 4 + a holds density s over its interval,
    so the coarse weights are w_k = e^{-s (t_k - t_K)} - e^{-s (t_{k+1} - t_K)}
    (t_S = far, K the first sample in the slab) and the cumulative pdf mass
    before sample k is 1 - e^{-s (t_k - t_K)} (k > K) plus 1e-5 (t_k - t_0).
    Each fine depth is t_k + (u - c_k) / (c_{k+1} - c_k) delta_k on that
    normalised cumulative c."""
    a, s = 0.85, 1.7
    spec = dict(TINY, n_coarse=16, n_fine=24, jitter=jitter)

    def field(sp, P, x, d):
        x = np.asarray(x, dtype=np.float64)
        sigma = np.where(x[:, 2] <= -a, s, 0.0)
        return sigma, np.full((x.shape[0], 3), 0.5)

    monkeypatch.setattr(mcl, "map_eval", field)
    o, d = np.array([0.0, 0.0, 4.0]), np.array([0.0, 0.0, -1.0])
    seed, it, key = 17, 2, (3, 5)
    r = mcl.render_rays(spec, None, [(o, d)], [key], seed, it, keep_samples=True)
    near, far, S, Sf = spec["near"], spec["far"], spec["n_coarse"], spec["n_fine"]
    k_ = np.arange(S)
    xi = px.unit24(px.word_at(seed, it, px.S_JIT_COARSE, key[0], key[1], k_)) if jitter else np.zeros(S)
    tc = near + (k_ + xi) * (far - near) / S
    t_next = np.append(tc[1:], far)
    K = int(np.argmax(tc >= 4.0 + a))
    cum = np.where(k_ > K, 1.0 - np.exp(-s * (tc - tc[K])), 0.0) + 1e-5 * (tc - tc[0])
    total = 1.0 - math.exp(-s * (far - tc[K])) + 1e-5 * (far - tc[0])
    c = np.append(cum, total) / total
    m = np.arange(Sf)
    xf = px.unit24(px.word_at(seed, it, px.S_JIT_FINE, key[0], key[1], m)) if jitter else np.full(Sf, 0.5)
    u = (m + xf) / Sf
    kk = np.searchsorted(c, u, side="right") - 1
    tf = tc[kk] + (u - c[kk]) / (c[kk + 1] - c[kk]) * (t_next - tc)[kk]
    want = np.sort(np.concatenate([tc, tf]))
    assert np.allclose(r["t"][0], want, rtol=0, atol=1e-12)
    # most fine samples sit in the slab's first few intervals, none before 4 + a
    # except the floor's share
    assert (tf >= 4.0 + a - (far - near) / S).mean() > 0.9
    # the coarse-plus-fine composite integrates the slab exactly: A = 1 - e^{-s (far - t_first)}
    first = want[np.argmax(want >= 4.0 + a)]
    assert abs(r["A"][0] - (1.0 - math.exp(-s * (far - first)))) < 1e-12


# ----------------------------------------------------------------------------- chordal mean, det < 0

def _quat_rot(q):
    w, x, y, z = q
    return np.array([[w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z]])


def _davenport(M):
    """The rotation maximising tr(R^T M) over SO(3): R(q) is a quadratic form
    in the unit quaternion q, so tr(R(q)^T M) = q^T K q with K obtained by
    polarisation, and the maximiser is K's top eigenvector."""
    f = lambda q: float(np.sum(_quat_rot(q) * M))
    e = np.eye(4)
    K = np.zeros((4, 4))
    for a_ in range(4):
        K[a_, a_] = f(e[a_])
        for b_ in range(a_ + 1, 4):
            K[a_, b_] = K[b_, a_] = 0.5 * (f(e[a_] + e[b_]) - f(e[a_]) - f(e[b_]))
    vals, vecs = np.linalg.eigh(K)
    return _quat_rot(vecs[:, -1])


def test_chordal_mean_with_negative_determinant_matches_davenport():
    rng = np.random.default_rng(11)
    found = 0
    for _ in range(400):
        n = int(rng.integers(3, 7))
        R = [synth.haar_rotation(rng) for _ in range(n)]
        w = rng.random(n) + 0.05
        M = sum(wi * Ri for wi, Ri in zip(w, R)) / w.sum()
        sv = np.linalg.svd(M, compute_uv=False)
        if np.linalg.det(M) >= -1e-3 or min(sv[0] - sv[1], sv[1] - sv[2]) < 0.05:
            continue
        poses = np.zeros((n, 3, 4))
        poses[:, :, :3] = R
        poses[:, :, 3] = rng.standard_normal((n, 3))
        est = se3.pose_estimate(poses, w)
        Rd = _davenport(M)
        assert np.allclose(est[:, :3], Rd, atol=1e-10, rtol=0)
        assert abs(np.linalg.det(est[:, :3]) - 1.0) < 1e-12
        assert np.allclose(est[:, 3], (w[:, None] * poses[:, :, 3]).sum(0) / w.sum(), atol=1e-14)
        found += 1
        if found == 5:
            break
    assert found == 5


def test_chordal_mean_with_positive_determinant_matches_davenport():
    rng = np.random.default_rng(12)
    R0 = synth.haar_rotation(rng)
    R = [R0 @ se3.exp_se3(np.zeros(3), 0.6 * rng.standard_normal(3))[:, :3] for _ in range(6)]
    w = rng.random(6)
    poses = np.zeros((6, 3, 4))
    poses[:, :, :3] = R
    M = sum(wi * Ri for wi, Ri in zip(w, R)) / w.sum()
    assert np.linalg.det(M) > 0
    assert np.allclose(se3.pose_estimate(poses, w)[:, :3], _davenport(M), atol=1e-10, rtol=0)
