"""Pins of the oracle's BF16 configuration of the map (render.mlp_bf16):
bfloat16 rounding against an independent library conversion, its
ties-to-even cases, the two-part head weights, a map whose every operand and
activation is a bfloat16 number (where the configuration must agree with the
float64 map exactly), and a hand-worked network whose hidden unit lands on a
rounding tie.  CPU only."""
import math

import numpy as np
import pytest
import torch

from oracle import mcl, render as rd


def test_round_bf16_matches_library_conversion():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(200_000) * np.exp2(rng.integers(-60, 60, 200_000))).astype(np.float32)
    x = np.concatenate([x, np.float32([0.0, -0.0, 1.0, -3.5, 2.0 ** -126, 3.0e38])])
    lib = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(rd.round_bf16(x.astype(np.float64)), lib)


def test_round_bf16_ties_to_even_and_bound():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: the even neighbour is 1;
    # 1 + 3 2^-8 lies halfway between 1 + 2^-7 and 1 + 2^-6: the even one is 1 + 2^-6
    assert rd.round_bf16(1 + 2.0 ** -8) == 1.0
    assert rd.round_bf16(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6
    assert rd.round_bf16(-(1 + 3 * 2.0 ** -8)) == -(1 + 2.0 ** -6)
    assert rd.round_bf16(257.0) == 256.0 and rd.round_bf16(259.0) == 260.0
    assert rd.round_bf16(255.0) == 255.0          # 8 significant bits are exact
    x = np.random.default_rng(1).uniform(-100, 100, 10_000)
    assert np.all(np.abs(rd.round_bf16(x) - x) <= 2.0 ** -8 * np.abs(x))   # unit roundoff of 8 bits


def test_split_bf16_keeps_sixteen_bits():
    rng = np.random.default_rng(2)
    w = rng.standard_normal(10_000).astype(np.float32).astype(np.float64)
    s = rd.split_bf16(w)
    assert np.all(np.abs(s - w) <= 2.0 ** -16 * np.abs(w))
    # both parts are bfloat16 numbers
    hi = rd.round_bf16(w)
    assert np.array_equal(rd.round_bf16(s - hi), s - hi)
    v = np.array([1.0 + 2.0 ** -12, -3.0 - 2.0 ** -10])   # 16 significant bits or fewer
    assert np.array_equal(rd.split_bf16(v), v)


def _small_spec(dir_width=0):
    return dict(n_layers=2, width=4, skip_layer=-1, L_xyz=0, L_dir=0, dir_width=dir_width)


def _params(spec, fill):
    parts = []
    for name, o, i in rd.layer_shapes(spec):
        W, b = fill(name, o, i)
        parts += [np.asarray(W, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64)]
    return np.concatenate(parts).astype(np.float32)


@pytest.mark.parametrize("dir_width", [0, 4])
def test_bf16_map_equals_float64_map_on_bfloat16_numbers(dir_width):
    # weights in {-1, -1/2, 0, 1/2, 1}, inputs with a few bits: every
    # pre-activation is a short dyadic number, so no rounding happens
    spec = _small_spec(dir_width)
    rng = np.random.default_rng(3)
    P = rd.unpack(spec, _params(spec, lambda n, o, i: (rng.integers(-2, 3, (o, i)) / 2.0,
                                                       rng.integers(-4, 5, o) / 4.0)))
    x = rng.integers(-16, 17, (50, 3)) / 8.0
    d = rng.integers(-8, 9, (50, 3)) / 8.0
    s64, c64 = rd.mlp(spec, P, x, d)
    s16, c16 = rd.mlp_bf16(spec, P, x, d)
    assert np.array_equal(s64, s16) and np.array_equal(c64, c16)


def test_bf16_map_hand_worked_rounding_tie():
    # inputs 129, 128, 130 are bfloat16 numbers (8 significant bits); unit 0
    # of layer 0 adds x0 + x1, layer 1 passes unit 0 on, and the density head
    # reads it with weight 1 + 2^-12 (kept whole by the two-part head weight)
    # and bias -250.  129 + 128 = 257 lies halfway between the bfloat16
    # numbers 256 and 258 and rounds to the even one, 256; 129 + 130 = 259
    # rounds to 260; the float64 map keeps 257 and 259
    spec = _small_spec()

    def fill(name, o, i):
        W, b = np.zeros((o, i)), np.zeros(o)
        if name == "h0":
            W[0, 0] = W[0, 1] = 1.0
        elif name == "h1":
            W[0, 0] = 1.0
        elif name == "sigma":
            W[0, 0] = 1.0 + 2.0 ** -12
            b[0] = -250.0
        return W, b

    P = rd.unpack(spec, _params(spec, fill))
    d = np.array([[0.0, 0.0, -1.0], [0.0, 0.0, -1.0]])
    x = np.array([[129.0, 128.0, 0.0], [129.0, 130.0, 0.0]])
    s16, _ = rd.mlp_bf16(spec, P, x, d)
    s64, _ = rd.mlp(spec, P, x, d)
    sp = lambda z: z + math.log1p(math.exp(-z))
    w = 1.0 + 2.0 ** -12
    assert abs(s16[0] - sp(256.0 * w - 250.0)) < 1e-12 and abs(s16[1] - sp(260.0 * w - 250.0)) < 1e-12
    assert abs(s64[0] - sp(257.0 * w - 250.0)) < 1e-12 and abs(s64[1] - sp(259.0 * w - 250.0)) < 1e-12


def test_bf16_configuration_through_the_renderer():
    # the update takes the BF16 map when the spec says so, and the result
    # stays within bfloat16's reach of the float64 map (relative 2^-8 per
    # operand over a few layers) on a smooth small map
    from paper_2406_12202_amd import synth
    s = synth.spec("small")
    p = synth.map_params(s, 5)
    cam = synth.camera("small")
    poses = synth.particles("small", 5, N=2)
    img = synth.observation("small", 5)
    a = mcl.update_particles(s, p, img, cam, 1, 4, poses, seed=1, it=1)
    b = mcl.update_particles(dict(s, precision="bf16"), p, img, cam, 1, 4, poses, seed=1, it=1)
    dC = np.abs(a["C"] - b["C"]).max()
    assert 0 < dC < 0.05
