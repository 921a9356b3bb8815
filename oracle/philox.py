"""Philox4x32-10 counter-based generator, written from its published definition.

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11 (the Philox-4x32 round and Weyl key
schedule, 10 rounds).  The random draws of the MCL update (query pixels,
stratified jitter, fine-sample jitter, motion noise, resampling offset) are all
taken from this generator under a fixed keying so that an independent
implementation on another device reproduces the same draws bit for bit.

Keying (shared specification, not shared code):
  key     = (seed & 0xffffffff, seed >> 32)
  counter = (c0, c1, iter & 0xffffffff, (stream << 24) | group)
The streams and the meaning of (c0, c1, group) are listed in STREAMS.
"""
import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF

# stream tags (the top byte of counter word 3)
S_PIX = 1        # query pixel j:           c0 = j,  c1 = 0, group 0, word 0
S_JIT_COARSE = 2  # coarse sample k of ray (i, j): c0 = i, c1 = j, group k // 4, word k % 4
S_JIT_FINE = 3   # fine sample m of ray (i, j):   c0 = i, c1 = j, group m // 4, word m % 4
S_MOTION = 4     # motion noise of particle i:    c0 = i, c1 = 0, groups 0 and 1
S_RESAMPLE = 5   # resampling offset:             c0 = 0, c1 = 0, group 0, word 0

STREAMS = {"pix": S_PIX, "jit_coarse": S_JIT_COARSE, "jit_fine": S_JIT_FINE,
           "motion": S_MOTION, "resample": S_RESAMPLE}


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox-4x32 rounds.  Arguments are integers or uint arrays (any
    shape, broadcast together); returns four uint64 arrays holding 32-bit words.
    One round: (hi0, lo0) = M0 * x0, (hi1, lo1) = M1 * x2,
    x <- (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0); the key is bumped by the Weyl
    constants between rounds."""
    x0, x1, x2, x3 = (np.asarray(v, dtype=np.uint64) & np.uint64(MASK)
                      for v in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & np.uint64(MASK)
    k1 = np.asarray(k1, dtype=np.uint64) & np.uint64(MASK)
    m = np.uint64(MASK)
    s32 = np.uint64(32)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(W0)) & m
            k1 = (k1 + np.uint64(W1)) & m
        p0 = np.uint64(M0) * x0          # < 2^64, exact in uint64
        p1 = np.uint64(M1) * x2
        hi0, lo0 = p0 >> s32, p0 & m
        hi1, lo1 = p1 >> s32, p1 & m
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def draw_words(seed, it, stream, c0, c1, group):
    """The four 32-bit words of one generator call (uint64 arrays)."""
    seed = int(seed)
    c3 = (np.uint64(stream) << np.uint64(24)) | np.asarray(group, dtype=np.uint64)
    return philox4x32_10(c0, c1, int(it) & MASK, c3, seed & MASK, (seed >> 32) & MASK)


def word_at(seed, it, stream, c0, c1, index):
    """Word number ``index`` of a stream where consecutive indices fill the four
    words of group index // 4 in order."""
    index = np.asarray(index, dtype=np.uint64)
    words = draw_words(seed, it, stream, c0, c1, index >> np.uint64(2))
    sel = (index & np.uint64(3)).astype(np.int64)
    return np.choose(sel, words)


def unit24(word):
    """Uniform in [0, 1): the top 24 bits of a word times 2^-24 (exact in fp32)."""
    return (np.asarray(word, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) * 2.0 ** -24


def unit_open(word):
    """Uniform in (0, 1): (word + 1/2) * 2^-32 (exact in fp64)."""
    return (np.asarray(word, dtype=np.uint64).astype(np.float64) + 0.5) * 2.0 ** -32
