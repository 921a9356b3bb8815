"""Multi-resolution grid map in float64: test infrastructure only (the checker
for the GPU grid-map kernel).

Sec. IV-B of the paper localises in a multi-scale grid map (Zip-NeRF) instead
of the plain NeRF MLP.  This is a restatement of the multiresolution hash
encoding of Instant-NGP (Mueller et al., 2022), the grid Zip-NeRF builds on,
with a tiny MLP; Zip-NeRF's anti-aliased multisampling is not part of it (a
reading recorded with the design notes).  Definitions:

  box        the map covers [-bound, bound]^3; u = (x + bound) / (2 bound);
             points with any u outside [0, 1] have sigma = 0 and colour 0
  levels     l = 0..L-1 with resolution N_l = floor(N_min b^l + 1e-6),
             b = exp((ln N_max - ln N_min) / (L - 1)) (b = 1 when L = 1; the
             1e-6 keeps N_{L-1} = N_max against rounding)
  vertex     p = u N_l, corner c = floor(p) + (i, j, k), weight
             prod over axes of (1 - |p - c|)
  index      (N_l + 1)^3 <= T: dense, c_0 + c_1 (N_l + 1) + c_2 (N_l + 1)^2;
             otherwise the spatial hash (c_0 * 1 xor c_1 * 2654435761 xor
             c_2 * 805459861) mod 2^32 mod T
  features   per level the trilinear blend of the F = 2 table entries of the
             8 corners; the 2L features are ordered level by level
  network    z = W2 relu(W1 f + b1) + b2 (64 hidden, 16 outputs),
             sigma = softplus(z_0);
             rgb = sigmoid(W4 relu(W3 [z, gamma(d)] + b3) + b4) (64 hidden)
  parameters tables: L x T x 2 float32 (level-major); mlp flat float32:
             W1 (64 x 2L), b1, W2 (16 x 64), b2, W3 (64 x (16 + in_d)), b3,
             W4 (3 x 64), b4, in_d = 3 + 6 L_dir
"""
import numpy as np

from . import render as rd

PRIMES = (1, 2654435761, 805459861)
HIDDEN = 64
GEO = 16


def resolutions(spec):
    L = spec["levels"]
    if L == 1:
        return [int(spec["n_min"])]
    b = np.exp((np.log(spec["n_max"]) - np.log(spec["n_min"])) / (L - 1))
    return [int(np.floor(spec["n_min"] * b ** l + 1e-6)) for l in range(L)]


def mlp_shapes(spec):
    in_d = 3 + 6 * spec["L_dir"]
    return [("W1", HIDDEN, 2 * spec["levels"]), ("W2", GEO, HIDDEN), ("W3", HIDDEN, GEO + in_d), ("W4", 3, HIDDEN)]


def n_mlp_params(spec):
    return sum(o * i + o for _, o, i in mlp_shapes(spec))


def unpack(spec, tables, mlp):
    T = 1 << spec["log2_table"]
    tab = np.asarray(tables, dtype=np.float32).astype(np.float64).reshape(spec["levels"], T, 2)
    flat = np.asarray(mlp, dtype=np.float32).astype(np.float64)
    P, pos = {"tables": tab}, 0
    for name, o, i in mlp_shapes(spec):
        P[name] = (flat[pos:pos + o * i].reshape(o, i), flat[pos + o * i:pos + o * i + o])
        pos += o * i + o
    if pos != flat.size:
        raise ValueError("mlp parameter count %d != %d" % (flat.size, pos))
    return P


def vertex_index(c, N, T):
    """Table index of integer vertex coordinates c (n, 3) at resolution N."""
    c = np.asarray(c, dtype=np.int64)
    if (N + 1) ** 3 <= T:
        return c[:, 0] + c[:, 1] * (N + 1) + c[:, 2] * (N + 1) ** 2
    h = np.zeros(c.shape[0], dtype=np.uint64)
    for a in range(3):
        h ^= (c[:, a].astype(np.uint64) * np.uint64(PRIMES[a])) & np.uint64(0xFFFFFFFF)
    return (h % np.uint64(T)).astype(np.int64)


def encode(spec, P, x):
    """Features (n, 2L) of points x (n, 3) and the inside-box mask."""
    x = np.asarray(x, dtype=np.float64)
    B = spec["bound"]
    u = (x + B) / (2.0 * B)
    inside = np.all((u >= 0.0) & (u <= 1.0), axis=1)
    u = np.clip(u, 0.0, 1.0)
    T = 1 << spec["log2_table"]
    feats = []
    for l, N in enumerate(resolutions(spec)):
        p = u * N
        c0 = np.minimum(np.floor(p), N - 1).astype(np.int64)     # p = N lies in the last cell
        f = np.zeros((x.shape[0], 2))
        for corner in range(8):
            off = np.array([(corner >> a) & 1 for a in range(3)])
            c = c0 + off
            w = np.prod(1.0 - np.abs(p - c), axis=1)
            f += w[:, None] * P["tables"][l][vertex_index(c, N, T)]
        feats.append(f)
    return np.concatenate(feats, axis=1), inside


def mlp(spec, P, x, d):
    """sigma (n,) and rgb (n, 3) of the grid map at points x seen along d."""
    f, inside = encode(spec, P, x)
    W1, b1 = P["W1"]
    W2, b2 = P["W2"]
    W3, b3 = P["W3"]
    W4, b4 = P["W4"]
    z = np.maximum(f @ W1.T + b1, 0.0) @ W2.T + b2
    sigma = rd.softplus(z[:, 0])
    gd = rd.posenc(d, spec["L_dir"])
    rgb = rd.sigmoid(np.maximum(np.concatenate([z, gd], axis=1) @ W3.T + b3, 0.0) @ W4.T + b4)
    sigma = np.where(inside, sigma, 0.0)
    rgb = np.where(inside[:, None], rgb, 0.0)
    return sigma, rgb
