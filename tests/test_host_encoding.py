"""Host check of the band-0 sin/cos of the bf16 encoding (sincospi_enc in the
MFMA kernels' shared header): its polynomial coefficients are read from the
source and the function is replayed in float32 arithmetic (each fused
multiply-add rounded once), then compared with sin(pi x) and cos(pi x) in
float64.  A mistyped coefficient or a wrong quarter-turn rotation moves the
result by far more than the bar.
"""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_2406_12202_amd", "csrc", "mfma_util.h")

f32 = np.float32


def _coefficients():
    src = open(HEADER).read()
    body = src[src.index("void sincospi_enc("):]
    body = body[:body.index("\n}\n")]
    vals = [float.fromhex(h) for h in re.findall(r"-?0x1\.[0-9a-f]+p[-+]\d+", body)]
    assert len(vals) == 10, vals
    return [f32(v) for v in vals[:5]], [f32(v) for v in vals[5:]]


def _fma(a, b, c):
    # float32 operands: the product is exact in float64, the sum rounds once
    return f32(np.float64(a) * np.float64(b) + np.float64(c))


def _sincospi(x, S, C):
    x = f32(x)
    j = f32(np.rint(np.float64(x) + np.float64(x)))
    r = _fma(j, f32(-0.5), x)
    z = f32(r * r)
    ps = _fma(z, S[0], S[1])
    for k in (2, 3, 4):
        ps = _fma(z, ps, S[k])
    sr = f32(r * ps)
    pc = _fma(z, C[0], C[1])
    for k in (2, 3, 4):
        pc = _fma(z, pc, C[k])
    cr = _fma(z, pc, f32(1.0))
    q = int(j)
    a, b = (cr, sr) if q & 1 else (sr, cr)
    return (-a if q & 2 else a), (-b if (q + 1) & 2 else b)


def test_band0_sincospi_error():
    S, C = _coefficients()
    rng = np.random.default_rng(7)
    xs = np.concatenate([rng.uniform(-12.0, 12.0, 20000), np.linspace(-2.0, 2.0, 4001),
                         np.array([0.0, 0.25, -0.25, 0.5, -0.5, 0.75, 1.0, -1.0, 1.5, 11.75])]).astype(np.float32)
    worst = 0.0
    for x in xs:
        s, c = _sincospi(x, S, C)
        xd = np.float64(x)
        worst = max(worst, abs(np.float64(s) - np.sin(np.pi * xd)), abs(np.float64(c) - np.cos(np.pi * xd)))
    print("largest error %.3e" % worst)
    assert worst <= 2.0 ** -23   # one float32 ulp of 1 (measured 8.4e-8)


def test_band0_quarter_turns_exact():
    """At multiples of 1/2 the reduction leaves r = 0: the values are exact."""
    S, C = _coefficients()
    for k in range(-8, 9):
        s, c = _sincospi(k / 2.0, S, C)
        assert float(s) == (0.0, 1.0, 0.0, -1.0)[k % 4] and float(c) == (1.0, 0.0, -1.0, 0.0)[k % 4], k
