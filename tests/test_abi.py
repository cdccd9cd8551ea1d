"""The C-ABI library loads, exports every declared entry point and validates
arguments before touching a GPU (runs without one)."""

import ctypes as C
import json
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pixvod.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pixvod_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["pixvod_create", "pixvod_set_keyframe", "pixvod_track", "pixvod_destroy",
              "pixvod_get_state", "pixvod_set_state"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2606_03989_amd as pv
    L = pv.lib()
    for n in declared_functions():
        assert hasattr(L, n), n
    # and the binding wraps each of them
    assert set(declared_functions()) == set(pv._SIGNATURES)


def test_default_params_are_the_papers():
    import paper_2606_03989_amd as pv
    with open(os.path.join(ROOT, "tests", "golden", "paper_hyperparameters.json")) as f:
        g = json.load(f)["values"]
    p = pv.default_params()
    for k in ("sigma_D", "sigma_P", "sigma_R", "sigma_N", "huber_k"):
        assert np.float32(getattr(p, k)) == np.float32(g[k])
    assert p.kf_max_frames == 150 and p.damping == 0.0


def _create(H, W, K, params=None):
    import paper_2606_03989_amd as pv
    h = C.c_void_p()
    Kc = None if K is None else pv.Intrinsics(*K)
    rc = pv.lib().pixvod_create(H, W, None if Kc is None else C.byref(Kc),
                                None if params is None else C.byref(params), C.byref(h))
    return rc, h


def test_argument_validation_precedes_device_use():
    import paper_2606_03989_amd as pv
    K = (30.0, 30.0, 16.0, 12.0)
    assert _create(1, 32, K)[0] == pv.EINVAL
    assert _create(24, 0, K)[0] == pv.EINVAL
    assert _create(24, 32, None)[0] == pv.EINVAL
    assert _create(24, 32, (0.0, 30.0, 16.0, 12.0))[0] == pv.EINVAL
    bad = pv.default_params(sigma_R=-1.0)
    assert _create(24, 32, K, bad)[0] == pv.EINVAL
    bad = pv.default_params(huber_k=float("nan"))
    assert _create(24, 32, K, bad)[0] == pv.EINVAL
    # context-free calls report through the thread-local message
    assert _create(1, 32, K)[0] == pv.EINVAL
    assert b"H and W" in pv.lib().pixvod_last_error(None)
    assert _create(24, 32, (0.0, 30.0, 16.0, 12.0))[0] == pv.EINVAL
    assert b"intrinsics" in pv.lib().pixvod_last_error(None)
    assert pv.lib().pixvod_create(24, 32, C.byref(pv.Intrinsics(*K)), None, None) == pv.EINVAL
    assert b"out_ctx" in pv.lib().pixvod_last_error(None)
    # NULL-context calls
    assert pv.lib().pixvod_track(None, None, 0, 1, None) == pv.EINVAL
    assert pv.lib().pixvod_set_keyframe(None, None, None, 0) == pv.EINVAL
    assert pv.lib().pixvod_iterate(None, 1) == pv.EINVAL
    assert pv.lib().pixvod_destroy(None) == pv.OK


def test_no_gpu_reports_enodev():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_2606_03989_amd as pv
    rc, h = _create(24, 32, (30.0, 30.0, 16.0, 12.0))
    assert rc == pv.ENODEV and not h.value
    with pytest.raises(pv.PixvodError) as e:
        pv.Tracker(24, 32, (30.0, 30.0, 16.0, 12.0))
    assert e.value.code == pv.ENODEV


def test_version_string():
    import paper_2606_03989_amd as pv
    assert "gfx950" in pv.version()
