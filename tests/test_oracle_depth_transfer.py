"""Pins of the oracle's keyframe depth transfer (depth propagation, Sec. 3.3;
re-anchoring, Sec. 3.5): identity motion leaves the depths, an axial motion of
a fronto-parallel plane shifts them by the motion, and on random depths and a
random pose the result equals a brute-force splat written independently here
(every candidate per target pixel listed, nearest FP32 depth kept)."""

import math

import numpy as np

import oracle
import synth


def _with_state(p, tau, ell):
    cam = p["cam"]
    o = oracle.Oracle(oracle.config_for_camera(cam, init_inv_depth=0.5))
    o.set_keyframe(p["I_s"], p["normals_s"])
    st = o.get_state()
    st[..., :6] = tau
    st[..., 6] = ell
    o.set_state(st)
    o.track(p["I_t"], 0)                  # the pose estimate is the mean pixel pose
    return o


def test_identity_motion_keeps_depths():
    p = synth.tiny_pair(0)
    cam = p["cam"]
    ell = np.random.default_rng(0).uniform(-0.5, 0.8, (cam.H, cam.W))
    o = _with_state(p, np.zeros(6), ell)
    o.transfer_depth()
    got = o.get_state()[..., 6]
    # every pixel lands on itself; depths are compared and stored at FP32
    np.testing.assert_allclose(got, np.log(np.exp(ell).astype(np.float32).astype(np.float64)), rtol=0, atol=1e-12)


def test_axial_motion_of_a_plane():
    p = synth.tiny_pair(0)
    cam = p["cam"]
    d, tz = 2.0, 0.5
    o = _with_state(p, np.array([0, 0, 0, 0, 0, tz]), np.full((cam.H, cam.W), math.log(d)))
    o.transfer_depth()
    got = o.get_state()[..., 6]
    new = math.log(float(np.float32(d + tz)))
    # the plane recedes and its image shrinks towards the principal point: the
    # central pixels receive it at depth d + tz, the border keeps depth d
    u0, v0 = int(cam.cx), int(cam.cy)
    assert abs(got[v0, u0] - new) < 1e-12
    assert np.all(np.abs(got[v0 - 3:v0 + 4, u0 - 3:u0 + 4] - new) < 1e-12)
    assert abs(got[0, 0] - math.log(d)) < 1e-12 and abs(got[-1, -1] - math.log(d)) < 1e-12
    frac = float(np.mean(np.abs(got - new) < 1e-12))
    assert 0.5 < frac < 0.8            # about (d / (d + tz))^2 = 0.64 of the image


def test_random_depths_equal_brute_force_splat():
    p = synth.tiny_pair(1)
    cam = p["cam"]
    rng = np.random.default_rng(3)
    ell = rng.uniform(-0.3, 1.2, (cam.H, cam.W))
    xi = np.array([0.01, -0.02, 0.015, 0.08, -0.05, 0.1])
    o = _with_state(p, xi, ell)
    o.transfer_depth()
    got = o.get_state()[..., 6]
    # brute force: every source pixel's candidate, listed per target
    T = oracle.se3_exp(xi)
    cand = {}
    for v in range(cam.H):
        for u in range(cam.W):
            dd = math.exp(ell[v, u])
            P = np.array([dd * (u - cam.cx) / cam.fx, dd * (v - cam.cy) / cam.fy, dd])
            Q = T[:3, :3] @ P + T[:3, 3]
            if Q[2] <= 0:
                continue
            ju = math.floor(cam.fx * Q[0] / Q[2] + cam.cx + 0.5)
            jv = math.floor(cam.fy * Q[1] / Q[2] + cam.cy + 0.5)
            if 0 <= ju < cam.W and 0 <= jv < cam.H:
                cand.setdefault((jv, ju), []).append(np.float32(Q[2]))
    ref = ell.copy()
    for (jv, ju), zs in cand.items():
        ref[jv, ju] = math.log(float(min(zs)))
    assert any(len(z) > 1 for z in cand.values())      # occlusions happen
    assert len(cand) < cam.H * cam.W                   # and holes
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_transfer_needs_a_tracked_frame():
    p = synth.tiny_pair(0)
    o = oracle.Oracle(oracle.config_for_camera(p["cam"]))
    o.set_keyframe(p["I_s"], p["normals_s"])
    try:
        o.transfer_depth()
        raise AssertionError("expected an error")
    except RuntimeError:
        pass
