"""One MCL update on a NeRF map in float64 (Alg. 1, Eq. 3, Eq. 6).

``update_particles`` runs the per-particle loop of Alg. 1: prediction, the
downscaled observation, rendering of B query pixels per particle at scale R,
the uncertainty-weighted photometric score of Eq. 6 and the normalised weights
of Eq. 3.  ``resample`` is the draw loop of Alg. 1 (systematic, with integer
thresholds so that any exact implementation returns identical indices).

Readings of points the paper leaves open (each is a named choice, listed with
the design notes): Eq. 6's garbled exponent is the square; E_j is the squared
L2 norm over RGB; one query-pixel set per update, shared by all particles and
drawn with replacement; S_i is floored at 1e-12 before the logarithm; the
log-likelihood is l_i = 4 (ln B - ln S_i), so w_i is proportional to
(B / S_i)^4 exactly.
"""
import math
import numpy as np

from . import grid as gr
from . import philox as px
from . import proposal as pr
from . import render as rd
from . import se3

FINE_FLOOR = 1e-5      # pdf mass added per unit length before fine placement
SCORE_FLOOR = 1e-12    # floor of S_i


# ----------------------------------------------------------------------------
# random draws (Philox4x32-10 keyed as documented in oracle.philox)

def pixel_indices(seed, it, B, n_pix):
    """p_j = floor(word0 * n_pix / 2^32), j = 0..B-1 (flat index v * W + u)."""
    w = px.word_at(seed, it, px.S_PIX, np.arange(B), 0, 0)
    return [(int(x) * int(n_pix)) >> 32 for x in w]


def coarse_t(spec, seed, it, i, j):
    """Stratified samples t_k = near + (k + xi_k) (far - near) / S_c."""
    S = spec["n_coarse"]
    k = np.arange(S)
    if spec["jitter"]:
        xi = px.unit24(px.word_at(seed, it, px.S_JIT_COARSE, i, j, k))
    else:
        xi = np.zeros(S)
    return spec["near"] + (k + xi) * ((spec["far"] - spec["near"]) / S)


def fine_u(spec, seed, it, i, j):
    """u_m = (m + xi'_m) / S_f (xi' = 1/2 without jitter)."""
    S = spec["n_fine"]
    m = np.arange(S)
    if spec["jitter"]:
        xi = px.unit24(px.word_at(seed, it, px.S_JIT_FINE, i, j, m))
    else:
        xi = np.full(S, 0.5)
    return (m + xi) / S


def motion_twist(seed, it, i, sigma_t, sigma_r):
    """Gaussian twist (rho, phi) ~ N(0, diag(sigma_t^2 I, sigma_r^2 I)) by
    Box-Muller on pairs of (0,1) uniforms: g = sqrt(-2 ln u1) (cos, sin)(2 pi u2)."""
    w = np.concatenate([px.draw_words(seed, it, px.S_MOTION, i, 0, g) for g in (0, 1)])
    u = px.unit_open(w)
    g = []
    for a in range(3):
        r = math.sqrt(-2.0 * math.log(u[2 * a]))
        g.append(r * math.cos(2.0 * math.pi * u[2 * a + 1]))
        g.append(r * math.sin(2.0 * math.pi * u[2 * a + 1]))
    rho = sigma_t * np.array(g[0:3])
    phi = sigma_r * np.array(g[3:6])
    return rho, phi


# ----------------------------------------------------------------------------
# prediction (Sec. III-A: x_t = x_{t-1} * O_t * Exp(delta))

def predict(pose, motion, sigma_t, sigma_r, seed, it, i):
    pose = np.asarray(pose, dtype=np.float64).reshape(3, 4)
    O = np.eye(4)[:3] if motion is None else np.asarray(motion, dtype=np.float64).reshape(3, 4)
    rho, phi = motion_twist(seed, it, i, sigma_t, sigma_r)
    return se3.compose(se3.compose(pose, O), se3.exp_se3(rho, phi))


# ----------------------------------------------------------------------------
# rendering of one particle's query rays

def unpack_map(spec, params):
    """Map parameters as the map type needs them: the NeRF MLP's flat vector,
    or, for a grid map (spec["map_type"] == "grid", Sec. IV-B), the pair
    (tables, mlp) of oracle.grid."""
    if spec.get("map_type") == "grid":
        return gr.unpack(spec, params[0], params[1])
    return rd.unpack(spec, params)


def map_eval(spec, P, x, d):
    """sigma and rgb of the map at points x seen along d; spec["precision"] ==
    "bf16" evaluates the NeRF map in its BF16 configuration (render.mlp_bf16),
    otherwise in float64."""
    if spec.get("map_type") == "grid":
        return gr.mlp(spec, P, x, d)
    if spec.get("precision") == "bf16":
        return rd.mlp_bf16(spec, P, x, d)
    return rd.mlp(spec, P, x, d)


def render_rays(spec, P, rays, keys, seed, it, proposal=None, keep_samples=False):
    """Render rays [(o, d)] whose random streams are keyed by (i, j) = keys[r].
    Fine samples (n_fine > 0) come from hierarchical sampling on the coarse
    weights, or, when ``proposal`` (flat proposal parameters) is given, from
    the proposal network's histogram.  Returns per-ray colour C, opacity A,
    z_trans, z_opaque, F and the densities at the two crossings."""
    B = len(rays)
    tc = [coarse_t(spec, seed, it, i, j) for (i, j) in keys]
    # coarse map queries for all rays in one batch
    X = np.concatenate([o[None, :] + t[:, None] * d[None, :] for (o, d), t in zip(rays, tc)])
    Dd = np.concatenate([np.repeat(d[None, :], t.size, 0) for (o, d), t in zip(rays, tc)])
    sig_c, rgb_c = map_eval(spec, P, X, Dd)
    Sc = spec["n_coarse"]
    far = spec["far"]
    ts, sigs, rgbs = [], [], []
    if spec["n_fine"] > 0:
        if proposal is not None:
            Q = pr.unpack(proposal)
            O = np.array([o for o, _ in rays])
            Dr = np.array([d for _, d in rays])
            hist, _ = pr.forward(Q, pr.features(O, Dr))
            tf = [pr.place(hist[r], spec["near"], far, fine_u(spec, seed, it, i, j))
                  for r, (i, j) in enumerate(keys)]
        else:
            tf = []
            for r, (i, j) in enumerate(keys):
                s = slice(r * Sc, (r + 1) * Sc)
                w, _, _, _ = rd.composite(tc[r], sig_c[s], rgb_c[s], far)
                mass = w + FINE_FLOOR * rd.deltas(tc[r], far)
                tf.append(rd.sample_pdf(tc[r], mass, far, fine_u(spec, seed, it, i, j)))
        Xf = np.concatenate([o[None, :] + t[:, None] * d[None, :] for (o, d), t in zip(rays, tf)])
        Df = np.concatenate([np.repeat(d[None, :], t.size, 0) for (o, d), t in zip(rays, tf)])
        sig_f, rgb_f = map_eval(spec, P, Xf, Df)
        Sf = spec["n_fine"]
        for r in range(B):
            sc, sf = slice(r * Sc, (r + 1) * Sc), slice(r * Sf, (r + 1) * Sf)
            t_all = np.concatenate([tc[r], tf[r]])
            order = np.argsort(t_all, kind="stable")   # ties: coarse first
            ts.append(t_all[order])
            sigs.append(np.concatenate([sig_c[sc], sig_f[sf]])[order])
            rgbs.append(np.concatenate([rgb_c[sc], rgb_f[sf]])[order])
    else:
        for r in range(B):
            s = slice(r * Sc, (r + 1) * Sc)
            ts.append(tc[r])
            sigs.append(sig_c[s])
            rgbs.append(rgb_c[s])
    # F of a ray whose opacity never reaches alpha: tau (inf of the empty set
    # is +inf), or far - near under spec["empty_ray"] == "span"
    empty = far - spec["near"] if spec.get("empty_ray") == "span" else None
    out = {k: np.zeros(B) for k in ("A", "z_trans", "z_opaque", "F", "sig_trans", "sig_opaque")}
    out["C"] = np.zeros((B, 3))
    if keep_samples:
        out["t"], out["w"] = [], []
    for r in range(B):
        w, logT, out["C"][r], out["A"][r] = rd.composite(ts[r], sigs[r], rgbs[r], far)
        out["z_trans"][r], out["z_opaque"][r] = rd.ray_quantiles(ts[r], sigs[r], logT, far, spec["alpha"])
        out["F"][r] = rd.uncertainty(out["z_trans"][r], out["z_opaque"][r], spec["tau"], empty)
        out["sig_trans"][r], out["sig_opaque"][r] = rd.crossing_densities(ts[r], sigs[r], logT, spec["alpha"])
        if keep_samples:
            out["t"].append(ts[r])
            out["w"].append(w)
    return out


def particle_rays(pose, pix, Wl, cam_l):
    fx, fy, cx, cy = cam_l
    return [rd.pixel_ray(pose, p % Wl, p // Wl, fx, fy, cx, cy) for p in pix]


def teacher_histograms(spec, params, O, D, seed, it):
    """Proposal training targets for rays (O[r], D[r]) from a full render of
    the map (streams keyed by (r, 0))."""
    P = unpack_map(spec, params)
    rays = [(np.asarray(o, dtype=np.float64), np.asarray(d, dtype=np.float64)) for o, d in zip(O, D)]
    r = render_rays(spec, P, rays, [(k, 0) for k in range(len(rays))], seed, it, keep_samples=True)
    return np.array([pr.teacher_histogram(t, w, spec["near"], spec["far"], A)
                     for t, w, A in zip(r["t"], r["w"], r["A"])])


def score(obs, C, F, B):
    """Eq. 6: E_j = |I(p_j) - C_j|^2 summed over RGB, S = sum_j E_j F_j,
    l = 4 (ln B - ln max(S, 1e-12)), i.e. w = (B / S)^4 in log form."""
    E = ((np.asarray(obs) - C) ** 2).sum(-1)
    S = float((E * F).sum())
    if math.isnan(S):
        return E, S, math.nan
    return E, S, 4.0 * (math.log(B) - math.log(max(S, SCORE_FLOOR)))


def normalise(loglik):
    """w_i = exp(l_i - m) / sum_k exp(l_k - m), m = max_k l_k (Eq. 3: weights
    normalised to [0, 1]).  Non-finite l_i get weight 0; if none is finite the
    set is degenerate and all weights are 0."""
    ll = np.asarray(loglik, dtype=np.float64)
    ok = np.isfinite(ll)
    w = np.zeros_like(ll)
    if not ok.any():
        return w
    m = ll[ok].max()
    e = np.where(ok, np.exp(np.where(ok, ll - m, 0.0)), 0.0)
    return e / e.sum()


def update_particles(spec, params, image, cam, inv_R, B, poses, motion=None,
                     sigma_t=0.0, sigma_r=0.0, seed=0, it=0, subset=None, proposal=None):
    """One weighting pass of Alg. 1 over the particles ``subset`` (default all).

    spec   : map/renderer settings (see oracle.render); params: flat float32 map
    image  : H x W x 3 observation; cam = (W, H, fx, fy, cx, cy) at full size
    inv_R  : level factor s, R_t = 1/s; intrinsics become R K (Sec. III-C)
    poses  : (N, 3, 4) particle poses x_{t-1}
    proposal: flat proposal-network parameters: fine samples from its
           histogram instead of hierarchical sampling
    Returns per-particle predicted poses, log-likelihoods, normalised weights
    (over the subset), mean uncertainty, and per-ray renders."""
    P = unpack_map(spec, params)
    Wf, Hf, fx, fy, cx, cy = cam
    s = int(inv_R)
    img_l = rd.downscale(image, s)
    Hl, Wl = img_l.shape[:2]
    cam_l = (fx / s, fy / s, cx / s, cy / s)
    pix = pixel_indices(seed, it, B, Wl * Hl)
    obs = np.array([img_l[p // Wl, p % Wl] for p in pix])
    poses = np.asarray(poses, dtype=np.float64).reshape(-1, 3, 4)
    idx = range(poses.shape[0]) if subset is None else list(subset)
    out = {"index": list(idx), "pose": [], "loglik": [], "score": [], "uncert": [],
           "C": [], "A": [], "F": [], "E": [], "z_trans": [], "z_opaque": [],
           "sig_trans": [], "sig_opaque": [],
           "pix": pix, "obs": obs}
    for i in idx:
        x = predict(poses[i], motion, sigma_t, sigma_r, seed, it, i)
        r = render_rays(spec, P, particle_rays(x, pix, Wl, cam_l), [(i, j) for j in range(B)], seed, it,
                        proposal=proposal)
        E, S, ll = score(obs, r["C"], r["F"], B)
        out["pose"].append(x)
        out["loglik"].append(ll)
        out["score"].append(S)
        out["uncert"].append(float(r["F"].mean()))
        for key in ("C", "A", "F", "z_trans", "z_opaque", "sig_trans", "sig_opaque"):
            out[key].append(r[key])
        out["E"].append(E)
    for key in ("pose", "loglik", "score", "uncert", "C", "A", "F", "E", "z_trans", "z_opaque",
                "sig_trans", "sig_opaque"):
        out[key] = np.array(out[key])
    out["weight"] = normalise(out["loglik"])
    return out


# ----------------------------------------------------------------------------
# resampling (Alg. 1, draw loop): systematic, integer thresholds

def resample(weight, n_out, seed, it):
    """Draw n_out indices with probability proportional to weight.

    q_i = floor(w_i / w_max * 2^40) (w_i <= 0 or non-finite counts as 0),
    Q = sum q_i, r0 = word 0 of the resampling stream,
    theta_k = floor((k 2^32 + r0) Q / (n_out 2^32)),
    idx_k = the smallest i whose inclusive prefix sum of q exceeds theta_k.
    All sums are exact integers; the only floating-point step is one correctly
    rounded division per particle.  Returns None when Q = 0 (degenerate)."""
    wt = [float(w) if (math.isfinite(float(w)) and float(w) > 0.0) else 0.0 for w in weight]
    wmax = max(wt) if wt else 0.0
    if wmax <= 0.0:
        return None
    q = [int(math.floor(w / wmax * 2.0 ** 40)) for w in wt]
    Q = sum(q)
    if Q == 0:
        return None
    r0 = int(px.draw_words(seed, it, px.S_RESAMPLE, 0, 0, 0)[0])
    prefix = []
    acc = 0
    for x in q:
        acc += x
        prefix.append(acc)
    out = []
    for k in range(n_out):
        theta = ((k << 32) + r0) * Q // (n_out << 32)
        lo, hi = 0, len(prefix) - 1          # smallest i with prefix[i] > theta
        while lo < hi:
            mid = (lo + hi) // 2
            if prefix[mid] > theta:
                hi = mid
            else:
                lo = mid + 1
        out.append(lo)
    return out


def resample_at(weight, n_out, seed, it, ks):
    """The draws idx_k of resample() for the k in ks only, for particle sets
    too large for its pure-Python loops: the same q_i (one float64 division,
    an exact scaling by 2^40 and a floor per weight), the inclusive prefix as
    a uint64 cumulative sum (exact: fewer than 2^24 terms of at most 2^40
    keep every partial sum below 2^64), theta_k in Python integers, and the
    smallest i with prefix_i > theta_k by binary search (searchsorted to the
    right of equal keys).  Returns None when Q = 0."""
    w = np.asarray(weight, dtype=np.float64)
    assert w.size < 2 ** 24, "the uint64 prefix is exact below 2^24 weights"
    wt = np.where(np.isfinite(w) & (w > 0.0), w, 0.0)
    wmax = float(wt.max()) if wt.size else 0.0
    if wmax <= 0.0:
        return None
    q = np.floor(wt / wmax * 2.0 ** 40).astype(np.uint64)
    prefix = np.cumsum(q, dtype=np.uint64)
    Q = int(prefix[-1])
    if Q == 0:
        return None
    r0 = int(px.draw_words(seed, it, px.S_RESAMPLE, 0, 0, 0)[0])
    out = []
    for k in ks:
        theta = ((int(k) << 32) + r0) * Q // (n_out << 32)
        out.append(int(np.searchsorted(prefix, np.uint64(theta), side="right")))
    return out


# ----------------------------------------------------------------------------
# coarse-to-fine levels with 1-sigma rejection (Alg. 1 with per-iteration
# R_t, B_t, N_t; Sec. III-C)

def reject_1sigma(uncert, loglik):
    """Rejection at a 1-sigma uncertainty threshold (a reading; the paper's own
    rejection is the soft weighting of Eq. 6): with U_i the mean F of particle
    i's rays, particles with U_i > mean(U) + std(U) get log-likelihood -inf
    (weight 0).  mean and the population standard deviation run over the
    particles with finite U and finite l; the others are rejected too."""
    U = np.asarray(uncert, dtype=np.float64)
    ll = np.asarray(loglik, dtype=np.float64).copy()
    ok = np.isfinite(U) & np.isfinite(ll)
    if not ok.any():
        return np.full_like(ll, -np.inf), np.ones(ll.shape, dtype=bool)
    mu = U[ok].mean()
    sd = math.sqrt(((U[ok] - mu) ** 2).mean())
    rejected = ~ok | (U > mu + sd)
    ll[rejected] = -np.inf
    return ll, rejected


def update_levels(spec, params, image, cam, levels, poses, motion=None, sigma_t=0.0, sigma_r=0.0,
                  seed=0, it=0, reject=True, proposal=None):
    """One coarse-to-fine update: for level L = 0, 1, ... with (inv_R, B,
    n_out) = levels[L], the particle set is predicted, weighted with B rays
    at scale 1/inv_R (update_particles, iteration counter it + L), optionally
    1-sigma rejected, normalised, and resampled to n_out particles (iteration
    counter it + L) that carry on to the next level.  Returns the per-level
    records and the final resampled poses; the pose read-out is that of the
    last level's weighted set."""
    X = np.asarray(poses, dtype=np.float64).reshape(-1, 3, 4)
    recs = []
    for L, (inv_R, B, n_out) in enumerate(levels):
        o = update_particles(spec, params, image, cam, inv_R, B, X, motion, sigma_t, sigma_r, seed, it + L,
                             proposal=proposal)
        ll = o["loglik"]
        rejected = np.zeros(ll.shape, dtype=bool)
        if reject:
            ll, rejected = reject_1sigma(o["uncert"], o["loglik"])
        w = normalise(ll)
        idx = resample(w, n_out, seed, it + L)
        recs.append(dict(out=o, loglik=ll, rejected=rejected, weight=w, index=idx))
        if idx is None:
            return dict(levels=recs, pose=None, estimate=None)
        est = se3.pose_estimate(o["pose"], w)
        X = o["pose"][idx]
    return dict(levels=recs, pose=X, estimate=est)


# ----------------------------------------------------------------------------
# localisation loop with variance-triggered refinement (Sec. III-C)

def position_variance(poses, weight):
    """Spread of the particle set: sum_i w_i |t_i - t_bar|^2 / sum_i w_i with
    t_bar the weighted mean position (the trace of the weighted covariance of
    the 3D positions; w <= 0 or non-finite counts as 0).  NaN if no weight."""
    P = np.asarray(poses, dtype=np.float64).reshape(-1, 3, 4)
    w = np.asarray(weight, dtype=np.float64)
    w = np.where(np.isfinite(w) & (w > 0.0), w, 0.0)
    W = w.sum()
    if not W > 0.0:
        return math.nan
    t = P[:, :, 3]
    tbar = (w[:, None] * t).sum(0) / W
    return float((w * ((t - tbar) ** 2).sum(1)).sum() / W)


def localize(spec, params, image, cam, stages, n_iters, poses, motion=None, sigma_t=0.0, sigma_r=0.0,
             seed=0, proposal=None):
    """The localisation loop: stages = [(inv_R, B, N, delta[, noise]), ...].
    At every iteration t (counter t) the particle set is updated at the
    current stage's scale and ray count (update_particles) with prediction
    noise (noise sigma_t, noise sigma_r) (noise = 1 when not given), the pose
    is read out and the position variance of the weighted set measured; when
    the variance falls below the stage's delta the next stage begins (the
    last stage's delta is never used); then N particles of the (possibly new)
    stage are drawn (counter t).  Returns per-iteration records and the final
    set."""
    X = np.asarray(poses, dtype=np.float64).reshape(-1, 3, 4)
    s = 0
    recs = []
    for t in range(n_iters):
        inv_R, B, N, delta = stages[s][:4]
        k = stages[s][4] if len(stages[s]) > 4 else 1.0
        o = update_particles(spec, params, image, cam, inv_R, B, X, motion, k * sigma_t, k * sigma_r, seed, t,
                             proposal=proposal)
        var = position_variance(o["pose"], o["weight"])
        est = se3.pose_estimate(o["pose"], o["weight"]) if np.any(o["weight"] > 0) else None
        rec = dict(iter=t, stage=s, var=var, est=est, loglik=o["loglik"], weight=o["weight"])
        if s + 1 < len(stages) and var < delta:
            s += 1
        idx = resample(o["weight"], stages[s][2], seed, t)
        rec["index"] = idx
        recs.append(rec)
        if idx is None:
            return dict(steps=recs, pose=None)
        X = o["pose"][idx]
    return dict(steps=recs, pose=X)
