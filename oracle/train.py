"""Map training with the photometric loss (Eq. 2) in float64: test
infrastructure only (the checker for the GPU gradient kernel).

Eq. 2 sums the squared colour error of rendered rays against the colours of
known-pose images.  Reading for a minibatch optimiser: the mean over the
rays of the batch, L = (1/|R|) sum_r |C_hat(r) - C(r)|^2, so that the step
size of Adam does not depend on the batch size.  C_hat(r) is the coarse
render of Eq. 1 exactly as the localisation path computes it (render.mlp,
render.composite; stratified samples keyed (r, 0) at counter `it`), for maps
without a skip input and without a direction branch (the 4 x 64 map).

The gradient follows the chain rule through the quadrature of Eq. 1 and the
network:
  with tau_k = sigma_k delta_k, T_k = exp(-sum_{m<k} tau_m), w_k = T_k (1 - e^{-tau_k}),
  dC/dc_k = w_k,
  dC/dtau_k = T_{k+1} c_k - sum_{m>k} w_m c_m,
then softplus' = sigmoid for the density head, c (1 - c) for the colour head,
and the ReLU layers backwards.  Parameters are read in float64 without a
float32 rounding so that finite differences of the loss can pin the gradient.
"""
import numpy as np

from . import mcl
from . import render as rd


def _unpack64(spec, flat):
    flat = np.asarray(flat, dtype=np.float64)
    out, pos = {}, 0
    for name, o, i in rd.layer_shapes(spec):
        W = flat[pos:pos + o * i].reshape(o, i)
        pos += o * i
        b = flat[pos:pos + o]
        pos += o
        out[name] = (W, b)
    if pos != flat.size:
        raise ValueError("parameter count %d != %d" % (flat.size, pos))
    return out


def _check_spec(spec):
    if spec["dir_width"] != 0 or (0 < spec["skip_layer"] < spec["n_layers"]) or spec["n_fine"] != 0:
        raise ValueError("map training covers maps without skip input or direction branch, coarse samples only")


def photometric_loss(spec, params, O, D, target, seed, it):
    """L = mean over rays r of |C_hat(r) - target_r|^2 (Eq. 2); ray r's
    samples are keyed (r, 0) at counter it."""
    return photometric_loss_grad(spec, params, O, D, target, seed, it, grad=False)[0]


def photometric_loss_grad(spec, params, O, D, target, seed, it, grad=True):
    """(L, dL/dtheta) with the gradient in the flat parameter order."""
    _check_spec(spec)
    P = _unpack64(spec, params)
    O = np.asarray(O, dtype=np.float64).reshape(-1, 3)
    D = np.asarray(D, dtype=np.float64).reshape(-1, 3)
    tgt = np.asarray(target, dtype=np.float64).reshape(-1, 3)
    R = O.shape[0]
    S = spec["n_coarse"]
    far = spec["far"]
    t = np.stack([mcl.coarse_t(spec, seed, it, r, 0) for r in range(R)])         # R x S
    X = (O[:, None, :] + t[:, :, None] * D[:, None, :]).reshape(-1, 3)
    Dd = np.repeat(D, S, axis=0)
    # forward through the network, keeping what the backward pass needs
    gx = rd.posenc(X, spec["L_xyz"])
    gd = rd.posenc(Dd, spec["L_dir"])
    acts, pre = [gx], []
    h = gx
    for l in range(spec["n_layers"]):
        W, b = P["h%d" % l]
        z = h @ W.T + b
        pre.append(z)
        h = np.maximum(z, 0.0)
        acts.append(h)
    ws, bs = P["sigma"]
    zs = (h @ ws.T + bs)[:, 0]
    sigma = rd.softplus(zs)
    g_in = np.concatenate([h, gd], axis=-1)
    Wc, bc = P["rgb"]
    zc = g_in @ Wc.T + bc
    c = rd.sigmoid(zc)
    # quadrature of Eq. 1 per ray
    sig = sigma.reshape(R, S)
    col = c.reshape(R, S, 3)
    delta = np.stack([rd.deltas(t[r], far) for r in range(R)])
    tau = sig * delta
    logT = np.concatenate([np.zeros((R, 1)), -np.cumsum(tau, axis=1)], axis=1)   # R x (S + 1)
    T = np.exp(logT)
    w = T[:, :-1] * (-np.expm1(-tau))
    C = (w[:, :, None] * col).sum(1)
    err = C - tgt
    L = float((err ** 2).sum() / R)
    if not grad:
        return L, None
    gC = 2.0 * err / R                                                           # R x 3
    wc = w[:, :, None] * col
    suffix = np.cumsum(wc[:, ::-1, :], axis=1)[:, ::-1, :] - wc                   # sum over m > k
    dtau = ((T[:, 1:, None] * col - suffix) * gC[:, None, :]).sum(-1)            # R x S
    dsig = (dtau * delta).reshape(-1)
    dcol = (w[:, :, None] * gC[:, None, :]).reshape(-1, 3)
    dzs = dsig * rd.sigmoid(zs)
    dzc = dcol * c * (1.0 - c)
    G = {}
    G["sigma"] = (dzs[None, :] @ h, np.array([dzs.sum()]))
    G["rgb"] = (dzc.T @ g_in, dzc.sum(0))
    da = dzs[:, None] * ws + dzc @ Wc[:, :spec["width"]]
    for l in range(spec["n_layers"] - 1, -1, -1):
        dz = da * (pre[l] > 0.0)
        G["h%d" % l] = (dz.T @ acts[l], dz.sum(0))
        W, _ = P["h%d" % l]
        da = dz @ W
    flat = np.concatenate([np.concatenate([G[name][0].ravel(), G[name][1].ravel()])
                           for name, _, _ in rd.layer_shapes(spec)])
    return L, flat


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015), t counted from 1; returns the new
    (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
