"""FP64 CPU oracle for the Fast Loc-NeRF particle update (arXiv 2406.12202).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything under ``oracle/``.  The
GPU product path never calls it, shares no code with it (no kernels, headers,
helpers, tables or constant generators) and must fail loudly when its HIP
library is missing instead of falling back here.

The oracle is plain, slow and written to be checked against the paper by eye:

* ``philox``  -- the counter-based generator both sides implement from its
  published definition (Salmon et al., SC'11, Philox4x32-10).
* ``se3``     -- SE(3) exponential, composition, pose read-out (Sec. III-A,
  prediction step).
* ``render``  -- positional encoding, the radiance-field MLP, volume rendering
  (Eq. 1), the transparent/opaque depths (Eq. 5) and the uncertainty
  F = max(z_opaque - z_trans, tau) (Sec. III-B), hierarchical fine sampling,
  image downscaling (Alg. 1, downscale step).
* ``mcl``     -- one MCL weighting pass (Alg. 1, per-particle loop) with the
  particle rejection weighting of Eq. 6, the normalised weights of Eq. 3 and
  systematic resampling (Alg. 1, draw loop).
* ``proposal`` -- the learned proposal histogram network: teacher targets,
  forward, analytic backward and Adam (not in the paper; an extension).

Every floating-point quantity is float64 unless stated.  Parity status: every
function is pinned by ``tests/test_oracle_*.py`` against closed forms,
invariants, special cases and brute force; none is "parity unpinned".
"""
