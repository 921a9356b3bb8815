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
