"""Pins of the oracle's learned-proposal functions: the analytic gradient
against central finite differences, Adam's first step in closed form,
softmax and histogram invariants, placement special cases, and a
proposal-guided render of a constant map in closed form."""
import math

import numpy as np
import pytest

from oracle import mcl, philox as px, proposal as pr, render as rd
from paper_2406_12202_amd import synth


def _random_problem(n=7, seed=0):
    rng = np.random.default_rng(seed)
    P = {name: rng.standard_normal(shp) * (0.3 if name.startswith("W") else 0.1) for name, shp in pr.SHAPES}
    O = rng.uniform(-4, 4, (n, 3))
    D = rng.standard_normal((n, 3))
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    T = rng.random((n, pr.N_BINS)) ** 3
    T /= T.sum(1, keepdims=True)
    return P, pr.features(O, D), T


def test_backward_matches_central_differences():
    P, x, T = _random_problem()
    _, cache = pr.forward(P, x)
    G = pr.backward(P, cache, T)
    theta = pr.pack(P)
    g = pr.pack(G)
    rng = np.random.default_rng(1)
    idx = rng.choice(theta.size, 300, replace=False)
    h = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fp = pr.loss(pr.forward(pr.unpack(tp), x)[0], T)
        fm = pr.loss(pr.forward(pr.unpack(tm), x)[0], T)
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_layout_and_counts():
    assert pr.N_IN == 78 and pr.N_PARAMS == 64 * 78 + 64 + 64 * 64 + 64 + 32 * 64 + 32
    P, _, _ = _random_problem()
    assert np.array_equal(pr.pack(pr.unpack(pr.pack(P))), pr.pack(P))


def test_adam_first_step_closed_form():
    # m0 = v0 = 0, t = 1: mhat = g, vhat = g^2, so theta moves by lr g / (|g| + eps)
    rng = np.random.default_rng(2)
    th, g = rng.standard_normal(50), rng.standard_normal(50)
    new, m, v = pr.adam_step(th, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    assert np.allclose(new, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_softmax_and_forward_invariants():
    P, x, _ = _random_problem()
    p, _ = pr.forward(P, x)
    assert np.allclose(p.sum(1), 1.0, atol=1e-15) and np.all(p > 0)
    P2 = dict(P)
    P2["b3"] = P["b3"] + 3.7          # a common shift of the logits changes nothing
    assert np.allclose(pr.forward(P2, x)[0], p, atol=1e-15)


def test_teacher_histogram_special_cases():
    near, far = 2.0, 6.0
    t = near + np.arange(64) * 4.0 / 64
    w = np.zeros(64)
    w[21] = 0.7                       # all weight at depth t[21] -> bin floor(21 / 2)
    h = pr.teacher_histogram(t, w, near, far, 0.7)
    assert h[10] == 1.0 and h.sum() == 1.0
    assert np.all(pr.teacher_histogram(t, w, near, far, 1e-4) == 1.0 / 32)
    rng = np.random.default_rng(3)
    w = rng.random(64)
    h = pr.teacher_histogram(t, w, near, far, 0.5)
    assert abs(h.sum() - 1.0) < 1e-15
    assert np.allclose(h, (w[0::2] + w[1::2]) / w.sum())


def test_placement_special_cases():
    near, far = 2.0, 6.0
    u = (np.arange(32) + 0.5) / 32
    out = pr.place(np.full(32, 1 / 32), near, far, u)
    assert np.allclose(out, near + u * 4.0, atol=1e-14)
    p = np.zeros(32)
    p[5] = 1.0
    out = pr.place(p, near, far, u)
    inside = ((out >= near + 5 * 0.125) & (out < near + 6 * 0.125)).mean()
    assert inside >= 0.96
    assert np.all(np.diff(out) >= 0)


@pytest.mark.parametrize("n_fine", [16, 32])
def test_proposal_guided_render_of_constant_map(n_fine):
    # constant density: the render integrates in closed form from the first
    # sample of the merged list, which may be a proposal-placed fine sample
    s = synth.spec("small", n_fine=n_fine)
    flat = []
    sizes = [(o, i) for _, o, i in rd.layer_shapes(s)]
    for n, (o, i) in enumerate(sizes):
        flat.append(np.zeros(o * i))
        b = np.zeros(o)
        if n == s["n_layers"]:
            b[:] = 0.3
        flat.append(b)
    flat = np.concatenate(flat).astype(np.float32)
    sig = math.log1p(math.exp(np.float32(0.3)))
    Q = {name: np.zeros(shp) for name, shp in pr.SHAPES}      # uniform proposal
    rng = np.random.default_rng(4)
    O = rng.uniform(-1, 1, (5, 3))
    D = rng.standard_normal((5, 3))
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    seed, it = 7, 2
    r = mcl.render_rays(s, rd.unpack(s, flat), list(zip(O, D)), [(k, 0) for k in range(5)], seed, it,
                        proposal=pr.pack(Q))
    near, far = s["near"], s["far"]
    for k in range(5):
        tc0 = near + px.unit24(px.word_at(seed, it, px.S_JIT_COARSE, k, 0, 0)) * (far - near) / s["n_coarse"]
        tf0 = near + px.unit24(px.word_at(seed, it, px.S_JIT_FINE, k, 0, 0)) / n_fine * (far - near)
        A = 1 - math.exp(-sig * (far - min(tc0, tf0)))
        assert abs(r["A"][k] - A) < 1e-13
