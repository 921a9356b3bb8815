"""NeRF map evaluation and volume rendering in float64 (Sec. III-A and III-B).

Map: F_NeRF(x, d) -> (c, sigma) (Sec. III-A), realised as the positional
encoding gamma and a ReLU MLP.  The paper only says "basic NeRF model"; the
layout below (identity term prepended to the encoding, pi in the frequencies,
optional skip input, optional direction branch) is the reading recorded with
the build's design notes.

Flat parameter order (float32 on input, read exactly as float64), for a map
with D hidden layers of width Wd, encodings of size in_x = 3 + 6 L_xyz and
in_d = 3 + 6 L_dir:
  for l in 0..D-1:  W_l (Wd x in_l, row-major), b_l (Wd)
       in_0 = in_x; in_l = Wd + in_x when l == skip_layer (input [h_{l-1}, gamma(x)]);
       otherwise in_l = Wd
  sigma head:  w_s (1 x Wd), b_s (1)            sigma = softplus(w_s h_{D-1} + b_s)
  if dir_width > 0:
      feature: W_f (Wd x Wd), b_f (Wd)         f = W_f h_{D-1} + b_f (no activation)
      dir:     W_v (dir_width x (Wd + in_d)), b_v   g = relu(W_v [f, gamma(d)] + b_v)
      rgb:     W_c (3 x dir_width), b_c (3)    c = sigmoid(W_c g + b_c)
  else:
      rgb:     W_c (3 x (Wd + in_d)), b_c (3)  c = sigmoid(W_c [h_{D-1}, gamma(d)] + b_c)
"""
import numpy as np


def posenc(p, L):
    """gamma(p) = (p, sin(2^0 pi p), cos(2^0 pi p), ..., sin(2^{L-1} pi p),
    cos(2^{L-1} pi p)), each term a 3-vector; output width 3 + 6 L."""
    p = np.asarray(p, dtype=np.float64)
    parts = [p]
    for l in range(L):
        a = (2.0 ** l) * np.pi * p
        parts.append(np.sin(a))
        parts.append(np.cos(a))
    return np.concatenate(parts, axis=-1)


def layer_shapes(spec):
    """[(name, out, in)] in flat-parameter order."""
    D, Wd, skip = spec["n_layers"], spec["width"], spec["skip_layer"]
    in_x = 3 + 6 * spec["L_xyz"]
    in_d = 3 + 6 * spec["L_dir"]
    shapes = []
    for l in range(D):
        if l == 0:
            nin = in_x
        elif l == skip:
            nin = Wd + in_x
        else:
            nin = Wd
        shapes.append(("h%d" % l, Wd, nin))
    shapes.append(("sigma", 1, Wd))
    if spec["dir_width"] > 0:
        shapes.append(("feature", Wd, Wd))
        shapes.append(("dir", spec["dir_width"], Wd + in_d))
        shapes.append(("rgb", 3, spec["dir_width"]))
    else:
        shapes.append(("rgb", 3, Wd + in_d))
    return shapes


def n_params(spec):
    return sum(o * i + o for _, o, i in layer_shapes(spec))


def unpack(spec, flat):
    """Split the flat parameter vector into {name: (W, b)} float64 arrays."""
    flat = np.asarray(flat, dtype=np.float32).astype(np.float64)
    out, pos = {}, 0
    for name, o, i in layer_shapes(spec):
        W = flat[pos:pos + o * i].reshape(o, i)
        pos += o * i
        b = flat[pos:pos + o]
        pos += o
        out[name] = (W, b)
    if pos != flat.size:
        raise ValueError("parameter count %d != %d" % (flat.size, pos))
    return out


def softplus(z):
    """log(1 + e^z), evaluated stably."""
    z = np.asarray(z, dtype=np.float64)
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    """1 / (1 + e^{-z})."""
    z = np.asarray(z, dtype=np.float64)
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(-z))


def mlp(spec, P, x, d):
    """Evaluate the map at points x (n, 3) seen along unit directions d (n, 3).
    Returns sigma (n,) and rgb (n, 3)."""
    gx = posenc(x, spec["L_xyz"])
    gd = posenc(d, spec["L_dir"])
    h = gx
    for l in range(spec["n_layers"]):
        if l == spec["skip_layer"] and l > 0:
            h = np.concatenate([h, gx], axis=-1)
        W, b = P["h%d" % l]
        h = np.maximum(h @ W.T + b, 0.0)
    ws, bs = P["sigma"]
    sigma = softplus(h @ ws.T + bs)[:, 0]
    if spec["dir_width"] > 0:
        Wf, bf = P["feature"]
        f = h @ Wf.T + bf
        Wv, bv = P["dir"]
        g = np.maximum(np.concatenate([f, gd], axis=-1) @ Wv.T + bv, 0.0)
    else:
        g = np.concatenate([h, gd], axis=-1)
    Wc, bc = P["rgb"]
    rgb = sigmoid(g @ Wc.T + bc)
    return sigma, rgb


def round_bf16(x):
    """Nearest bfloat16 value (8 significant bits, ties to even; the float32
    exponent range): with x = m 2^e, 1/2 <= |m| < 1, the value
    rint(m 2^8) 2^(e - 8), where rint rounds halves to even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    e = np.maximum(e, -125)            # below 2^-126 the spacing stays 2^-133
    m = np.ldexp(x, -e)
    return np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)


def split_bf16(w):
    """A weight carried as two bfloat16 numbers: hi = bf16(w), lo = bf16(w - hi)."""
    hi = round_bf16(w)
    return hi + round_bf16(np.asarray(w, dtype=np.float64) - hi)


def mlp_bf16(spec, P, x, d):
    """The map in the BF16 configuration: every product of a hidden, feature
    or direction layer multiplies bfloat16 operands -- the encodings
    gamma(x), gamma(d), the layer's weights and the previous layer's output,
    each rounded to the nearest bfloat16 -- and sums them with the float32
    bias exactly (float32 accumulation on the device); each layer's output
    (after ReLU where the layer has one) is rounded to bfloat16 as the next
    layer's input.  The density and colour heads act on those bfloat16
    activations with weights carried as a pair of bfloat16 numbers
    (split_bf16).  softplus and sigmoid as in mlp."""
    r = round_bf16
    gx = r(posenc(x, spec["L_xyz"]))
    gd = r(posenc(d, spec["L_dir"]))
    h = gx
    for l in range(spec["n_layers"]):
        if l == spec["skip_layer"] and l > 0:
            h = np.concatenate([h, gx], axis=-1)
        W, b = P["h%d" % l]
        h = r(np.maximum(h @ r(W).T + b, 0.0))
    ws, bs = P["sigma"]
    sigma = softplus(h @ split_bf16(ws).T + bs)[:, 0]
    if spec["dir_width"] > 0:
        Wf, bf = P["feature"]
        f = r(h @ r(Wf).T + bf)
        Wv, bv = P["dir"]
        g = r(np.maximum(np.concatenate([f, gd], axis=-1) @ r(Wv).T + bv, 0.0))
    else:
        g = np.concatenate([h, gd], axis=-1)
    Wc, bc = P["rgb"]
    rgb = sigmoid(g @ split_bf16(Wc).T + bc)
    return sigma, rgb


def pixel_ray(pose, u, v, fx, fy, cx, cy):
    """Camera ray through pixel (u, v) of a pinhole camera with intrinsics
    (fx, fy, cx, cy) (Eq. 4: r(p, x) with intrinsics K).  OpenGL convention
    (x right, y up, looking along -z), pixel centres at +1/2:
    d_cam = ((u + 1/2 - cx)/fx, -(v + 1/2 - cy)/fy, -1), d = R d_cam / |R d_cam|,
    o = t.  The ray parameter is Euclidean distance along d."""
    pose = np.asarray(pose, dtype=np.float64).reshape(3, 4)
    dc = np.array([(u + 0.5 - cx) / fx, -(v + 0.5 - cy) / fy, -1.0])
    d = pose[:, :3] @ dc
    return pose[:, 3].copy(), d / np.linalg.norm(d)


def deltas(t, far):
    """Interval lengths of the Riemann sum: delta_k = t_{k+1} - t_k and
    delta_{S-1} = far - t_{S-1}; density is zero outside [t_0, far]."""
    t = np.asarray(t, dtype=np.float64)
    return np.append(t[1:], far) - t


def composite(t, sigma, rgb, far):
    """Eq. 1 as a Riemann sum with sigma and c constant on [t_k, t_k + delta_k):
    tau_k = sigma_k delta_k, log T_k = -sum_{m<k} tau_m,
    w_k = T_k (1 - e^{-tau_k}), C = sum_k w_k c_k, A = sum_k w_k = 1 - T_S.
    No background term (black background).  Returns w, logT (length S + 1), C, A."""
    sigma = np.asarray(sigma, dtype=np.float64)
    tau = sigma * deltas(t, far)
    logT = np.concatenate([[0.0], -np.cumsum(tau)])
    w = np.exp(logT[:-1]) * (-np.expm1(-tau))
    C = (w[:, None] * np.asarray(rgb, dtype=np.float64)).sum(0)
    A = float(w.sum())
    return w, logT, C, A


def ray_quantiles(t, sigma, logT, far, alpha):
    """Eq. 5 with the exact cumulative weight of piecewise-constant density:
    int_0^z T sigma ds = 1 - T(z).  z_trans = min{z : 1 - T(z) >= alpha} (the
    point where T first falls to 1 - alpha; +inf when it never does) and
    z_opaque = max{z : 1 - T(z) <= 1 - alpha} (the point where T falls to alpha;
    capped at far when it never does).  Inside interval k the transmittance is
    T_k e^{-sigma_k (z - t_k)}, so the crossing of level L is
    t_k + (log T_k - log L) / sigma_k."""
    t = np.asarray(t, dtype=np.float64)
    S = t.size
    l_trans = np.log1p(-alpha)
    l_opq = np.log(alpha)
    z_trans = np.inf
    for k in range(S):
        if logT[k + 1] <= l_trans:
            z_trans = t[k] + (logT[k] - l_trans) / sigma[k]
            break
    z_opaque = far
    for k in range(S):
        if logT[k + 1] < l_opq:
            z_opaque = t[k] + (logT[k] - l_opq) / sigma[k]
            break
    return z_trans, z_opaque


def crossing_densities(t, sigma, logT, alpha):
    """Density on the intervals where T crosses 1 - alpha and alpha (nan when
    it does not).  The crossing depths of ray_quantiles move by
    |log L| * eps / sigma under a relative change eps of all optical depths, so
    these densities give the conditioning of z_trans, z_opaque and F."""
    l_trans, l_opq = np.log1p(-alpha), np.log(alpha)
    st = so = np.nan
    for k in range(len(t)):
        if np.isnan(st) and logT[k + 1] <= l_trans:
            st = sigma[k]
        if logT[k + 1] < l_opq:
            so = sigma[k]
            break
    return st, so


def uncertainty(z_trans, z_opaque, tau, empty=None):
    """F = max(z_opaque - z_trans, tau) (Sec. III-B, below Eq. 6).  A ray that
    never becomes non-transparent (z_trans = inf of the empty set = +inf)
    gets F = tau; with ``empty`` given (the reading that such a ray has no
    transparent-to-opaque transition in the sampled span and is maximally
    uncertain, far - near) it gets F = empty."""
    if not np.isfinite(z_trans):
        return float(tau if empty is None else empty)
    return float(max(z_opaque - z_trans, tau))


def sample_pdf(t, mass, far, u):
    """Inverse-CDF placement on the piecewise-constant pdf that puts mass
    mass_k uniformly on [t_k, t_k + delta_k).  For each u in [0, 1): find the
    interval k with c_k <= u < c_{k+1} of the normalised cumulative masses and
    return t_k + (u - c_k) / (c_{k+1} - c_k) * delta_k."""
    t = np.asarray(t, dtype=np.float64)
    dl = deltas(t, far)
    mass = np.asarray(mass, dtype=np.float64)
    c = np.concatenate([[0.0], np.cumsum(mass)]) / mass.sum()
    out = np.empty(len(u))
    for m, um in enumerate(u):
        k = int(np.searchsorted(c, um, side="right")) - 1
        k = min(max(k, 0), t.size - 1)
        out[m] = t[k] + (um - c[k]) / (c[k + 1] - c[k]) * dl[k]
    return out


def downscale(img, s):
    """Box average of s x s pixel blocks (Alg. 1, downscale(I_t, R_t) with
    R_t = 1/s); img is H x W x 3."""
    img = np.asarray(img, dtype=np.float64)
    H, W, C = img.shape
    if H % s or W % s:
        raise ValueError("image size not divisible by the level factor")
    return img.reshape(H // s, s, W // s, s, C).mean(axis=(1, 3))
