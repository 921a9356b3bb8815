"""Host-side checks of the C-ABI library: it loads, exports every entry point
declared in include/fastloc.h, and rejects bad arguments before touching the
GPU.  No compute call is made, so these run without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2406_12202_amd import binding, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastloc.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(loc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libfastloc.so is not built (run __graft_entry__.build())")
    return binding.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "loc_init_map" in names and "loc_update_particles" in names and "loc_resample" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(binding.EXPORTS) == set(names)


def test_status_strings(lib):
    for s in (0, -1, -2, -3, -4, -5, -6, 42):
        assert lib.loc_status_str(s)
    assert lib.loc_status_str(binding.LOC_E_UNSUPPORTED) == b"unsupported map shape or precision"
    assert lib.loc_last_error(None) == b""


def _init(lib, spec, params, **over):
    d, keep = binding.map_desc(spec, params)
    for k, v in over.items():
        setattr(d, k, v)
    h = ctypes.c_void_p(1234)
    st = lib.loc_init_map(ctypes.byref(d), None, ctypes.byref(h))
    return st, h, keep


def test_init_rejects_bad_arguments_without_a_gpu(lib):
    s = synth.spec("small")
    p = synth.map_params(s, 0)
    assert lib.loc_init_map(None, None, None) == binding.LOC_E_ARG
    for over, want in [(dict(alpha=0.0), binding.LOC_E_ARG), (dict(alpha=0.5), binding.LOC_E_ARG),
                       (dict(tau=0.0), binding.LOC_E_ARG), (dict(far_=1.0), binding.LOC_E_ARG),
                       (dict(n_coarse=0), binding.LOC_E_ARG), (dict(n_coarse=257), binding.LOC_E_ARG),
                       (dict(n_fine=-1), binding.LOC_E_ARG), (dict(width=128), binding.LOC_E_UNSUPPORTED),
                       (dict(L_xyz=5), binding.LOC_E_UNSUPPORTED),
                       (dict(n_params=p.size - 1), binding.LOC_E_ARG)]:
        st, h, _ = _init(lib, s, p, **over)
        assert st == want, (over, st)
        assert h.value is None           # *out is cleared on failure
    d, _ = binding.map_desc(s, p)
    d.params = None
    assert lib.loc_init_map(ctypes.byref(d), None, ctypes.byref(ctypes.c_void_p())) == binding.LOC_E_ARG


def test_update_and_resample_reject_null_context(lib):
    cam = binding.Camera(W=64, H=64, fx=60.0, fy=60.0, cx=32.0, cy=32.0)
    assert lib.loc_update_particles(None, None, ctypes.byref(cam), 1, 1, 1, None, None, 0.0, 0.0, 0, 0,
                                    None, None, None, None) == binding.LOC_E_ARG
    assert lib.loc_resample(None, None, 1, 1, 0, 0, None) == binding.LOC_E_ARG
    assert lib.loc_resample_noalloc(None, None, 1, 1, 0, 0, None) == binding.LOC_E_ARG
    assert lib.loc_sync(None, None) == binding.LOC_E_ARG
    assert lib.loc_ray_outputs(None, None, None, None, None) == binding.LOC_E_ARG
    lib.loc_destroy(None)


def test_parameter_count_matches_documented_layout():
    # the documented flat-parameter layout gives these sizes for the two maps
    small = synth.spec("small")
    nerf = synth.spec("nerf")
    n_small = synth.map_params(small, 0).size
    n_nerf = synth.map_params(nerf, 0).size
    assert n_small == (39 * 64 + 64) + 3 * (64 * 64 + 64) + (64 + 1) + (79 * 3 + 3)
    assert n_nerf == ((63 * 256 + 256) + 4 * (65536 + 256) + (319 * 256 + 256) + 2 * (65536 + 256)
                      + (256 + 1) + (65536 + 256) + (283 * 128 + 128) + (128 * 3 + 3))
