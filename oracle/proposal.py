"""Learned proposal network in float64: teacher histograms, forward, analytic
backward, Adam and proposal-guided fine placement.

The paper renders with plain NeRF sampling (Sec. III-A, Eq. 1); this network
is an extension that places the fine samples of a ray from a predicted
32-bin density histogram instead of from a coarse render.  Definitions (the
readings are listed with the design notes):

  input      x = [gamma_6(o), gamma_6(d)]  (78 values; gamma as in render.posenc)
  network    h1 = relu(W1 x + b1) (64), h2 = relu(W2 h1 + b2) (64),
             z = W3 h2 + b3 (32), p = softmax(z)
  parameters flat float32 in the order W1 (64 x 78), b1, W2 (64 x 64), b2,
             W3 (32 x 64), b3
  teacher    h_b = sum of the compositing weights w_s of the full render whose
             sample depth t_s lies in bin b of 32 equal bins on [near, far),
             divided by sum_s w_s; uniform when the ray's opacity is < 1e-3
  loss       mean over rays of sum_b (p_b - h_b)^2
  optimiser  Adam (Kingma and Ba, 2015): m <- b1 m + (1 - b1) g,
             v <- b2 v + (1 - b2) g^2, theta <- theta - lr mhat / (sqrt(vhat) + eps)
  placement  pdf mass_b = 0.99 p_b + 0.01 / 32 on the bins, inverse CDF at
             u_m = (m + xi'_m) / S_f
"""
import numpy as np

from . import render as rd

N_BINS = 32
HIDDEN = 64
L_ENC = 6
N_IN = 2 * (3 + 6 * L_ENC)
SHAPES = [("W1", (HIDDEN, N_IN)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
          ("W3", (N_BINS, HIDDEN)), ("b3", (N_BINS,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
UNIFORM_MIX = 0.01
EMPTY_OPACITY = 1e-3


def unpack(flat):
    flat = np.asarray(flat, dtype=np.float64)
    if flat.size != N_PARAMS:
        raise ValueError("proposal parameter count %d != %d" % (flat.size, N_PARAMS))
    out, pos = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = flat[pos:pos + n].reshape(shp)
        pos += n
    return out


def pack(P):
    return np.concatenate([np.asarray(P[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def features(o, d):
    """x = [gamma_6(o), gamma_6(d)] for rays (n, 3) and (n, 3)."""
    return np.concatenate([rd.posenc(o, L_ENC), rd.posenc(d, L_ENC)], axis=-1)


def softmax(z):
    e = np.exp(z - z.max(axis=-1, keepdims=True))
    return e / e.sum(axis=-1, keepdims=True)


def forward(P, x):
    """Returns p and the intermediate values used by backward."""
    a1 = x @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ P["W3"].T + P["b3"]
    p = softmax(z)
    return p, dict(x=x, a1=a1, h1=h1, a2=a2, h2=h2, z=z, p=p)


def loss(p, target):
    return float(((p - target) ** 2).sum(axis=-1).mean())


def backward(P, cache, target):
    """Gradient of the mean squared histogram error, by the chain rule:
    dL/dp = 2 (p - h) / n; dL/dz = p * (dL/dp - sum_b p_b dL/dp_b) (softmax
    Jacobian); a linear layer y = W u + b passes dL/dW = dy^T u,
    dL/db = sum dy, dL/du = dy W; ReLU passes the gradient where its input
    is > 0."""
    n = target.shape[0]
    p = cache["p"]
    gp = 2.0 * (p - target) / n
    gz = p * (gp - (p * gp).sum(axis=-1, keepdims=True))
    G = {}
    G["W3"] = gz.T @ cache["h2"]
    G["b3"] = gz.sum(0)
    gh2 = gz @ P["W3"]
    ga2 = gh2 * (cache["a2"] > 0)
    G["W2"] = ga2.T @ cache["h1"]
    G["b2"] = ga2.sum(0)
    gh1 = ga2 @ P["W2"]
    ga1 = gh1 * (cache["a1"] > 0)
    G["W1"] = ga1.T @ cache["x"]
    G["b1"] = ga1.sum(0)
    return G


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of flat arrays (t counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def teacher_histogram(t, w, near, far, opacity):
    """Bin the compositing weights w (at sample depths t) into 32 equal bins
    of [near, far) and normalise; uniform when the ray is nearly empty."""
    if opacity < EMPTY_OPACITY:
        return np.full(N_BINS, 1.0 / N_BINS)
    b = np.floor((np.asarray(t) - near) / (far - near) * N_BINS).astype(int)
    b = np.clip(b, 0, N_BINS - 1)
    h = np.zeros(N_BINS)
    np.add.at(h, b, w)
    return h / h.sum()


def place(p, near, far, u):
    """Fine depths from the proposal pdf 0.99 p + 0.01 / 32 on equal bins."""
    mass = (1.0 - UNIFORM_MIX) * np.asarray(p, dtype=np.float64) + UNIFORM_MIX / N_BINS
    c = np.concatenate([[0.0], np.cumsum(mass)]) / mass.sum()
    width = (far - near) / N_BINS
    out = np.empty(len(u))
    for m, um in enumerate(u):
        b = int(np.searchsorted(c, um, side="right")) - 1
        b = min(max(b, 0), N_BINS - 1)
        out[m] = near + (b + (um - c[b]) / (c[b + 1] - c[b])) * width
    return out
