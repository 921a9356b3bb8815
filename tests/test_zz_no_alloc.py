"""The allocation-free resampling entry point (loc_resample_noalloc) against
loc_resample through the C ABI: bit-identical indices on two calls in a row,
the second with fewer weights (the fixed scratch keeps the first call's
prefix beyond the second's n_in), and the size limit."""
import numpy as np
import pytest

from oracle import mcl
from paper_2406_12202_amd import binding, synth

pytestmark = pytest.mark.gpu


def _weights(rng, n):
    w = rng.random(n) ** 6
    w[rng.random(n) < 0.1] = 0.0
    return w / w.sum()


def test_noalloc_resample_matches_resample_twice():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dev = torch.device("cuda", 0)
    s = synth.spec("small")
    c = binding.Context(s, synth.map_params(s, 0))
    rng = np.random.default_rng(7)
    for n_in, n_out, seed, it in ((300_000, 120_000, 11, 2), (4097, 5000, 11, 3)):
        w = _weights(rng, n_in)
        wd = torch.as_tensor(w, device=dev)
        a = c.loc_resample(wd, n_out, seed, it)
        b = c.loc_resample_noalloc(wd, n_out, seed, it)
        flags = c.loc_sync()
        assert flags == 0
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.array_equal(a, b), (n_in, n_out)
        ks = [0, 1, n_out // 2, n_out - 1]
        assert b[ks].tolist() == mcl.resample_at(w, n_out, seed, it, ks)
    c.close()


def test_noalloc_resample_limits_and_degenerate():
    import torch
    dev = torch.device("cuda", 0)
    s = synth.spec("small")
    c = binding.Context(s, synth.map_params(s, 0))
    big = torch.zeros(binding.LOC_NOALLOC_MAX_WEIGHTS + 1, dtype=torch.float64, device=dev)
    with pytest.raises(RuntimeError, match="loc_resample_noalloc"):
        c.loc_resample_noalloc(big, 4)
    # all-zero weights: indices -1 and the degenerate-resampling flag, as loc_resample
    z = torch.zeros(1000, dtype=torch.float64, device=dev)
    idx = c.loc_resample_noalloc(z, 16, 1, 1)
    assert c.loc_sync() == binding.FLAG_DEGENERATE_RESAMPLE
    assert (idx.cpu().numpy() == -1).all()
    # exactly at the limit: equal weights draw every particle once
    n = binding.LOC_NOALLOC_MAX_WEIGHTS
    u = torch.full((n,), 1.0 / n, dtype=torch.float64, device=dev)
    idx = c.loc_resample_noalloc(u, n, 5, 0)
    assert c.loc_sync() == 0
    assert np.array_equal(idx.cpu().numpy(), np.arange(n))
    c.close()
