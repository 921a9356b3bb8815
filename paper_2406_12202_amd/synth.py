"""Seeded synthetic inputs for the Fast Loc-NeRF particle update.

This module is the only code that both the GPU path's callers (tests, bench)
and the CPU oracle's callers use.  It holds none of the method's arithmetic:
it makes map parameters, camera poses, particle sets and observation images of
the shapes and distributions of the workloads, from numpy's seeded PCG64.

Workloads (the paper's LLFF/NeRF data and trained maps are not available; these
synthetic stand-ins have the same shapes):
  small    4x64 map, 64x64 image f=60, 32 particles on a radius-4 sphere with
           Haar-random rotation, 16 rays, 32 stratified samples in [2, 6]
  nerf     8x256 map (skip at layer 5, L=10/4, 128-wide direction branch),
           400x400 image f=555, 400 particles on the upper radius-4 hemisphere
           looking at the origin with a random yaw, 64 rays, 64 + 128 samples
  c2f      4x64 map, 800x800 image f=1110, levels 1/4, 1/2, 1 with
           16 / 64 / 256 rays and 1000 -> 300 -> 100 particles
  proposal nerf workload with 64 coarse + 32 proposal-placed fine samples
  large    8x256 map, 1008x756 forward-facing image f=815, 2000 particles
           within +-1 m / +-30 deg of the ground truth, 256 rays,
           64 + 32 samples, motion noise 0.02 m / 1 deg
"""
import math
import numpy as np

SMALL_MAP = dict(n_layers=4, width=64, skip_layer=-1, L_xyz=6, L_dir=2, dir_width=0)
NERF_MAP = dict(n_layers=8, width=256, skip_layer=5, L_xyz=10, L_dir=4, dir_width=128)
RENDER = dict(near=2.0, far=6.0, alpha=0.05, tau=0.1, jitter=1)

WORKLOADS = {
    "small": dict(map=SMALL_MAP, n_coarse=32, n_fine=0, W=64, H=64, f=60.0,
                  N=32, B=16, inv_R=1, particles="sphere", gt="sphere"),
    "nerf": dict(map=NERF_MAP, n_coarse=64, n_fine=128, W=400, H=400, f=555.0,
                 N=400, B=64, inv_R=1, particles="hemisphere", gt="hemisphere"),
    "c2f": dict(map=SMALL_MAP, n_coarse=32, n_fine=0, W=800, H=800, f=1110.0,
                N=1000, B=16, inv_R=4, particles="hemisphere", gt="hemisphere",
                levels=[(4, 16, 1000), (2, 64, 300), (1, 256, 100)]),
    "proposal": dict(map=NERF_MAP, n_coarse=64, n_fine=32, W=400, H=400, f=555.0,
                     N=400, B=64, inv_R=1, particles="hemisphere", gt="hemisphere"),
    "large": dict(map=NERF_MAP, n_coarse=64, n_fine=32, W=1008, H=756, f=815.0,
                  N=2000, B=256, inv_R=1, particles="forward", gt="forward",
                  sigma_t=0.02, sigma_r=math.radians(1.0), iterations=10),
}


def spec(workload, **over):
    """Flat map + renderer settings dict for a workload."""
    w = WORKLOADS[workload]
    s = dict(w["map"])
    s.update(RENDER)
    s.update(n_coarse=w["n_coarse"], n_fine=w["n_fine"])
    s.update(over)
    return s


def camera(workload):
    """(W, H, fx, fy, cx, cy) at full resolution, principal point at the centre."""
    w = WORKLOADS[workload]
    return (w["W"], w["H"], w["f"], w["f"], w["W"] / 2.0, w["H"] / 2.0)


def _shapes(s):
    """(out, in) of each weight matrix in flat-parameter order (the documented
    parameter format of the map)."""
    D, Wd, skip = s["n_layers"], s["width"], s["skip_layer"]
    in_x, in_d = 3 + 6 * s["L_xyz"], 3 + 6 * s["L_dir"]
    out = []
    for l in range(D):
        out.append((Wd, in_x if l == 0 else (Wd + in_x if l == skip else Wd)))
    out.append((1, Wd))
    if s["dir_width"] > 0:
        out += [(Wd, Wd), (s["dir_width"], Wd + in_d), (3, s["dir_width"])]
    else:
        out.append((3, Wd + in_d))
    return out


# density-head gain and bias per map size, chosen so that per-ray opacity spans
# [0, 1] and the transparent-to-opaque gap spans [tau, far - near]
DENSITY_INIT = {64: (10.0, 5.0), 256: (16.0, 12.0)}


# embedded solid: the density pre-activation gains gain * relu(radius - |x|_1)
SOLID = dict(gain=20.0, radius=1.5)


def map_params(s, seed, sigma_bias=None, band_decay=0.5, sigma_gain=None, solid=True):
    """Seeded random-init map parameters (float32, flat).

    Hidden weights are He-scaled N(0, 2/fan_in) with zero biases; the columns
    of the first layer (and of the skip input) that read the frequency-l
    encoding terms are scaled by band_decay**l so that the density field has
    both empty and opaque stretches instead of uniform fog; the density output
    weights are multiplied by sigma_gain and get bias sigma_bias.

    With ``solid`` (the default) the map also holds an opaque octahedron
    |x|_1 < 1.5 inside the random field: hidden units 0..5 of the first layer
    compute relu(+-x_c), unit 6 of the second layer computes
    relu(1.5 - sum of them) and passes through every later layer unchanged,
    and the density head adds 20 times it, so rays that reach the solid see a
    surface whose depth varies smoothly with the ray."""
    g0, b0 = DENSITY_INIT.get(s["width"], (1.0, 0.0))
    sigma_gain = g0 if sigma_gain is None else sigma_gain
    sigma_bias = b0 if sigma_bias is None else sigma_bias
    rng = np.random.default_rng(seed)
    in_x = 3 + 6 * s["L_xyz"]
    # per-column gain of an encoding block: identity terms 1, band l terms band_decay**l
    gx = np.ones(in_x)
    for l in range(s["L_xyz"]):
        gx[3 + 6 * l: 9 + 6 * l] = band_decay ** l
    parts = []
    shapes = _shapes(s)
    for n, (o, i) in enumerate(shapes):
        W = rng.standard_normal((o, i)) * math.sqrt(2.0 / i)
        if n == 0:
            W = W * gx[None, :]
        elif n == s["skip_layer"] and n < s["n_layers"]:
            W[:, s["width"]:] *= gx[None, :]
        b = np.zeros(o)
        if n == s["n_layers"]:          # sigma head
            W = W * sigma_gain
            b[:] = sigma_bias
        if solid:
            if n == 0:                  # units 0..5: relu(+x_c), relu(-x_c)
                W[:6, :] = 0.0
                for u in range(6):
                    W[u, u // 2] = 1.0 if u % 2 == 0 else -1.0
            elif n == 1:                # unit 6: relu(radius - |x|_1)
                W[6, :] = 0.0
                W[6, :6] = -1.0
                b[6] = SOLID["radius"]
            elif n < s["n_layers"]:     # unit 6 passes through
                W[6, :] = 0.0
                W[6, 6] = 1.0
            elif n == s["n_layers"]:    # density head
                W[0, 6] = SOLID["gain"]
        parts += [W.ravel(), b]
    return np.concatenate(parts).astype(np.float32)


def lookat(eye, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)):
    """Camera-to-world 3x4 [R | t] whose -z axis points from eye to target
    (OpenGL camera: x right, y up)."""
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    up = np.asarray(up, dtype=np.float64)
    if abs(f @ up) > 0.999:
        up = np.array([0.0, 1.0, 0.0])
    x = np.cross(f, up)
    x /= np.linalg.norm(x)
    y = np.cross(x, f)
    P = np.zeros((3, 4))
    P[:, 0], P[:, 1], P[:, 2], P[:, 3] = x, y, -f, eye
    return P


def haar_rotation(rng):
    """Uniformly random rotation (Shoemake's uniform unit quaternion)."""
    u1, u2, u3 = rng.random(3)
    a, b = math.sqrt(1 - u1), math.sqrt(u1)
    qx, qy = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    qz, qw = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qz * qw), 2 * (qx * qz + qy * qw)],
        [2 * (qx * qy + qz * qw), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qx * qw)],
        [2 * (qx * qz - qy * qw), 2 * (qy * qz + qx * qw), 1 - 2 * (qx * qx + qy * qy)]])


def _rotz(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _rot_exp(phi):
    th = np.linalg.norm(phi)
    if th < 1e-12:
        return np.eye(3)
    k = phi / th
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K


def _sphere_point(rng, upper=False):
    v = rng.standard_normal(3)
    v /= np.linalg.norm(v)
    if upper:
        v[2] = abs(v[2])
    return 4.0 * v


def gt_pose(workload, seed):
    kind = WORKLOADS[workload]["gt"]
    rng = np.random.default_rng([seed, 1])
    if kind == "forward":
        P = np.zeros((3, 4))
        P[:, :3] = np.eye(3)
        P[:, 3] = (0.0, 0.0, 4.0)
        return P
    return lookat(_sphere_point(rng, upper=(kind == "hemisphere")))


def particles(workload, seed, N=None, gt=None):
    """Initial particle poses (N, 3, 4) float64."""
    w = WORKLOADS[workload]
    N = w["N"] if N is None else N
    rng = np.random.default_rng([seed, 2])
    out = np.zeros((N, 3, 4))
    for i in range(N):
        if w["particles"] == "sphere":
            out[i, :, :3] = haar_rotation(rng)
            out[i, :, 3] = _sphere_point(rng)
        elif w["particles"] == "hemisphere":
            P = lookat(_sphere_point(rng, upper=True))
            out[i, :, :3] = _rotz(rng.uniform(-math.pi, math.pi)) @ P[:, :3]
            out[i, :, 3] = P[:, 3]
        else:  # forward: +-1 m per axis and +-30 deg per rotation-vector axis
            g = gt_pose(workload, seed) if gt is None else gt
            phi = np.radians(rng.uniform(-30.0, 30.0, 3))
            out[i, :, :3] = g[:, :3] @ _rot_exp(phi)
            out[i, :, 3] = g[:, 3] + rng.uniform(-1.0, 1.0, 3)
    return out


def observation(workload, seed, noise=0.01):
    """Procedural H x W x 3 float32 observation: a smooth colour field plus
    Gaussian pixel noise.  The weighting pass reads the image only through the
    downscaled query pixels, so its content sets no amount of work."""
    w = WORKLOADS[workload]
    H, W = w["H"], w["W"]
    rng = np.random.default_rng([seed, 3])
    v, u = np.meshgrid(np.arange(H) / H, np.arange(W) / W, indexing="ij")
    img = np.empty((H, W, 3))
    for c in range(3):
        a, b, ph = rng.uniform(0.5, 3.0), rng.uniform(0.5, 3.0), rng.uniform(0, 2 * math.pi)
        img[..., c] = 0.5 + 0.3 * np.sin(2 * math.pi * (a * u + b * v) + ph)
    img += noise * rng.standard_normal(img.shape)
    return img.astype(np.float32)


def add_noise(img, seed, noise=0.01):
    rng = np.random.default_rng([seed, 4])
    return (np.asarray(img, dtype=np.float64) + noise * rng.standard_normal(np.shape(img))).astype(np.float32)


def proposal_params(seed):
    """Seeded He-scaled initial parameters of the 78 -> 64 -> 64 -> 32 proposal
    network (flat float32: W1, b1, W2, b2, W3, b3), zero biases."""
    rng = np.random.default_rng([seed, 5])
    parts = []
    for o, i in ((64, 78), (64, 64), (32, 64)):
        parts += [rng.standard_normal((o, i)).ravel() * math.sqrt(2.0 / i), np.zeros(o)]
    return np.concatenate(parts).astype(np.float32)


def training_poses(workload, seed, n):
    """Poses for proposal training rays: the workload's particle distribution
    under a separate seed."""
    return particles(workload, seed + 7919, N=n)


def random_histograms(seed, n, bins=32):
    """Seeded random target histograms (rows sum to 1)."""
    rng = np.random.default_rng([seed, 6])
    h = rng.random((n, bins)) ** 4
    return (h / h.sum(1, keepdims=True)).astype(np.float32)


# ---------------------------------------------------------------------------
# Structured scene: a closed room (axis-aligned box) with a procedural texture
# on each of its six faces and eight textured pillars standing in front of the
# walls, seen from inside.  Training rays are rendered
# exactly (first face hit along the ray); a map trained on them has a valid
# region (inside the room) and an untrained one beyond its walls.

ROOM = dict(half=(3.5, 3.5, 2.5),            # room extent: |x| <= 3.5, |y| <= 3.5, |z| <= 2.5
            # floor-to-ceiling pillars (centre x, y, half width): depth steps in front of the walls
            pillars=((2.7, 2.7, 0.35), (-2.7, 2.7, 0.35), (2.7, -2.7, 0.35), (-2.7, -2.7, 0.35),
                     (3.1, 0.0, 0.25), (-3.1, 0.0, 0.25), (0.0, 3.1, 0.25), (0.0, -3.1, 0.25)),
            views=(0.75, 0.75, 0.25),        # training cameras: |x| <= 0.75, |y| <= 0.75, |z| <= 0.25
            pitch_deg=15.0,
            W=160, H=120, f=140.0)           # camera of the room workload
_FACE_BASE = np.array([[0.85, 0.35, 0.30], [0.30, 0.70, 0.40], [0.30, 0.40, 0.85],
                       [0.85, 0.75, 0.30], [0.60, 0.35, 0.75], [0.35, 0.75, 0.80]])


def room_camera():
    r = ROOM
    return (r["W"], r["H"], r["f"], r["f"], r["W"] / 2.0, r["H"] / 2.0)


def room_colour(p, face):
    """Texture of face `face` (0/1: x = -/+, 2/3: y = -/+, 4/5: z = -/+) at
    points p (n, 3): the face colour modulated by two crossed sinusoids of
    periods 2.5 to 5 units and a checker of 2-unit squares, values in
    [0.05, 0.95]."""
    p = np.asarray(p, dtype=np.float64)
    out = np.zeros((p.shape[0], 3))
    for fc in range(6):
        m = face == fc
        if not np.any(m):
            continue
        ax = fc // 2
        u, v = [p[m, a] for a in range(3) if a != ax]
        f1, f2 = 0.25 + 0.05 * fc, 0.35 - 0.03 * fc
        pat = 0.5 + 0.3 * np.sin(2 * math.pi * f1 * u + 0.7 * fc) * np.cos(2 * math.pi * f2 * v + fc)
        chk = ((np.floor(u / 2.0) + np.floor(v / 2.0)) % 2) * 0.3 - 0.15
        val = np.clip(pat + chk, 0.0, 1.0)
        base = _FACE_BASE[fc]
        out[m] = np.clip(0.05 + 0.9 * (val[:, None] * base + (1 - val[:, None]) * (1 - base) * 0.5), 0.05, 0.95)
    return out


def room_render(O, D, far=None):
    """Colour of the first room face hit by rays from inside (black beyond
    `far`, when given)."""
    O = np.asarray(O, dtype=np.float64).reshape(-1, 3)
    D = np.asarray(D, dtype=np.float64).reshape(-1, 3)
    half = np.array(ROOM["half"])
    with np.errstate(divide="ignore", invalid="ignore"):
        tp = np.where(D > 0, (half - O) / D, np.inf)
        tn = np.where(D < 0, (-half - O) / D, np.inf)
    t_ax = np.minimum(tp, tn)
    ax = np.argmin(t_ax, axis=1)
    t = t_ax[np.arange(O.shape[0]), ax]
    face = 2 * ax + (tp[np.arange(O.shape[0]), ax] <= tn[np.arange(O.shape[0]), ax]).astype(int)
    P = O + t[:, None] * D
    C = room_colour(P, face)
    # pillars: slab test in x and y (they span the full height)
    for q, (px, py, hw) in enumerate(ROOM["pillars"]):
        lo = np.array([px - hw, py - hw])
        hi = np.array([px + hw, py + hw])
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = (lo - O[:, :2]) / D[:, :2]
            t2 = (hi - O[:, :2]) / D[:, :2]
        tmin = np.nanmax(np.minimum(t1, t2), axis=1)
        tmax = np.nanmin(np.maximum(t1, t2), axis=1)
        hit = (tmin <= tmax) & (tmin > 0) & (tmin < t)
        if np.any(hit):
            t = np.where(hit, tmin, t)
            Ph = O[hit] + tmin[hit, None] * D[hit]
            u = Ph[:, 0] + Ph[:, 1]
            v = Ph[:, 2]
            stripe = 0.5 + 0.4 * np.sign(np.sin(2 * math.pi * (0.8 * v + 0.3 * q)))
            base = _FACE_BASE[(q + 2) % 6]
            C[hit] = np.clip(0.1 + 0.8 * (stripe[:, None] * (1 - base) + (1 - stripe[:, None]) * base * 0.7)
                             + 0.05 * np.sin(2 * math.pi * 0.5 * u)[:, None], 0.05, 0.95)
    if far is not None:
        C[t > far] = 0.0
    return C


def room_pose(rng):
    """A camera inside the view box looking horizontally (random yaw, pitch
    within +-ROOM['pitch_deg'])."""
    r = ROOM
    eye = rng.uniform(-1.0, 1.0, 3) * np.array(r["views"])
    yaw = rng.uniform(-math.pi, math.pi)
    pitch = math.radians(rng.uniform(-r["pitch_deg"], r["pitch_deg"]))
    fwd = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    return lookat(eye, eye + fwd)


def room_rays(seed, n_views, rays_per_view, far=6.0):
    """Training rays of the room: n_views random cameras, rays_per_view random
    pixels each; returns O, D (float32, n x 3, unit D) and the exact colours
    (float32), shuffled."""
    rng = np.random.default_rng([seed, 11])
    W, H, fx, fy, cx, cy = room_camera()
    O, D = [], []
    for _ in range(n_views):
        P = room_pose(rng)
        u = rng.integers(0, W, rays_per_view) + 0.5
        v = rng.integers(0, H, rays_per_view) + 0.5
        dc = np.stack([(u - cx) / fx, -(v - cy) / fy, -np.ones(rays_per_view)], 1)
        d = dc @ P[:, :3].T
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        O.append(np.repeat(P[None, :, 3], rays_per_view, 0))
        D.append(d)
    O, D = np.concatenate(O), np.concatenate(D)
    C = room_render(O, D, far)
    perm = rng.permutation(O.shape[0])
    return O[perm].astype(np.float32), D[perm].astype(np.float32), C[perm].astype(np.float32)


def room_image(pose, far=6.0):
    """Exact H x W x 3 image of the room from `pose` (pixel centres as the
    update's rays)."""
    W, H, fx, fy, cx, cy = room_camera()
    P = np.asarray(pose, dtype=np.float64).reshape(3, 4)
    v, u = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    dc = np.stack([(u - cx) / fx, -(v - cy) / fy, -np.ones_like(u)], -1).reshape(-1, 3)
    d = dc @ P[:, :3].T
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    C = room_render(np.repeat(P[None, :, 3], d.shape[0], 0), d, far)
    return C.reshape(H, W, 3).astype(np.float32)


def room_particles(seed, N, gt, spread_m, spread_deg):
    """N poses around gt: position offsets uniform in +-spread_m per axis (half
    that vertically), rotation vector uniform in +-spread_deg per axis."""
    rng = np.random.default_rng([seed, 12])
    out = np.zeros((N, 3, 4))
    for i in range(N):
        phi = np.radians(rng.uniform(-spread_deg, spread_deg, 3))
        out[i, :, :3] = gt[:, :3] @ _rot_exp(phi)
        out[i, :, 3] = gt[:, 3] + rng.uniform(-1.0, 1.0, 3) * np.array([spread_m, spread_m, 0.5 * spread_m])
    return out


def room_map_init(seed):
    """Initial parameters of the 4x64 map for training on the room (He-scaled
    weights, zero biases; no built-in solid)."""
    return map_params(spec("small"), seed, solid=False)


# ---------------------------------------------------------------------------
# Multi-resolution grid map (16 levels of 2^19 two-feature entries, resolutions
# 16 .. 2048 over [-4, 4]^3, 64-wide tiny MLP), the second map type.

GRID_MAP = dict(map_type="grid", levels=16, log2_table=19, n_min=16, n_max=2048, bound=4.0, L_dir=2)


def grid_spec(n_coarse=64, n_fine=128, **over):
    s = dict(GRID_MAP)
    s.update(RENDER)
    s.update(n_coarse=n_coarse, n_fine=n_fine)
    s.update(over)
    return s


def grid_params(s, seed, feature_scale=0.5):
    """Seeded grid tables (L x T x 2 float32, N(0, feature_scale^2) rounded to
    half-precision values, which the grid map stores exactly) and tiny-MLP
    parameters (He-scaled weights, zero biases; the density output's weights
    x3 and bias -1 so that sigma spans empty and opaque stretches)."""
    rng = np.random.default_rng([seed, 31])
    T = 1 << s["log2_table"]
    tables = (feature_scale * rng.standard_normal((s["levels"], T, 2))).astype(np.float16).astype(np.float32)
    in_d = 3 + 6 * s["L_dir"]
    parts = []
    for name, o, i in (("W1", 64, 2 * s["levels"]), ("W2", 16, 64), ("W3", 64, 16 + in_d), ("W4", 3, 64)):
        W = rng.standard_normal((o, i)) * math.sqrt(2.0 / i)
        b = np.zeros(o)
        if name == "W2":
            W[0] *= 3.0
            b[0] = -1.0
        parts += [W.ravel(), b]
    return tables.ravel(), np.concatenate(parts).astype(np.float32)
