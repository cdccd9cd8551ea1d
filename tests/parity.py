"""Shared helpers of the parity tests: workloads, state layout conversion and
the agreement measures.

Parity bar:
  pose (mean per-pixel se(3) vector)   |xi_gpu - xi_oracle|_inf <= 1e-5
  inverse depth                         relative RMS and 99th percentile of
                                        |rho_gpu - rho_or| / rho_or <= 1e-4
The state is FP32 on the GPU and FP64 in the oracle. The iteration amplifies
small differences (the FP64 oracle itself turns a 1e-12 perturbation of the
log-depths into ~1e-6 pose differences within two frames on the textured
sequences), so:
  * every iteration is checked teacher-forced: oracle and GPU start from the
    same FP32 state and all 123 planes are compared after one iteration, the
    maximum and the 99.9th percentile of the plane-relative error bounded by
    1e-5 or by twice the oracle's own change under an FP32-resolution
    perturbation of that state, whichever is larger;
  * free-running runs bound pose, and the RMS, 99th percentile and maximum of
    the inverse-depth error, by the fixed bar or by twice the oracle's own
    spread over the same horizon, whichever is larger.
The spread is the largest difference between the oracle's run and runs of its
own at the GPU's storage precision: the starting log-depths moved at FP32
resolution, and the oracle's storage emulation (every new message rounded to
FP32 before the update uses it, as the GPU keeps messages in FP32 state planes
between their computation and their use, and the state rounded after every
iteration), from the same start and from moved starts. Where the iteration is
well conditioned (the tiny pair at sigma_P = 0.1) the spread is ~1e-8 and the
fixed bar applies; at the paper's sigma_P = 1 the storage precision alone moves
the oracle's own 50-iteration result by up to ~3e-3 in pose.
"""

from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

import oracle
import synth
from synth.scenes import SEQUENCE_CONFIGS, make_sequence_scene, render_sequence_frame, sequence_poses

POSE_TOL = 1e-5
DEPTH_TOL = 1e-4

# factor strengths per workload: the paper's leaf values except the prior,
# which on the flat grid is the weakest decade value whose early iterations
# stay stable (the paper's selection rule for the prior)
SEQ_PARAMS = {
    "ppa256": dict(sigma_P=0.01, huber_k=400.0),
    "vga": dict(sigma_P=0.01, huber_k=10.0),
    "diff320": dict(sigma_P=0.01, huber_k=10.0),
}


def to_oracle(state: np.ndarray) -> np.ndarray:
    """(123, H, W) float32 exchange layout -> (H, W, 123) float64."""
    return np.ascontiguousarray(np.transpose(state.astype(np.float64), (1, 2, 0)))


def from_oracle(state: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.transpose(state, (2, 0, 1)).astype(np.float32))


def tree_to_oracle(state):
    """Quadtree exchange layout ((42, H, W), (141, NT)) float32 -> the
    oracle's ((H, W, 42), (NT, 141)) float64."""
    pix, nodes = state
    return (np.ascontiguousarray(np.transpose(pix.astype(np.float64), (1, 2, 0))),
            np.ascontiguousarray(nodes.astype(np.float64).T))


def tree_from_oracle(state):
    pix, nodes = state
    return (np.ascontiguousarray(np.transpose(pix, (2, 0, 1)).astype(np.float32)),
            np.ascontiguousarray(nodes.T.astype(np.float32)))


def depth_agreement(rho_gpu: np.ndarray, rho_or: np.ndarray) -> Dict[str, float]:
    e = np.abs(rho_gpu.astype(np.float64) - rho_or) / np.abs(rho_or)
    return dict(rms=float(np.sqrt(np.mean(e * e))), p99=float(np.percentile(e, 99)),
                max=float(e.max()), frac_over=float(np.mean(e > DEPTH_TOL)))


def pose_agreement(xi_gpu, xi_or) -> float:
    return float(np.abs(np.asarray(xi_gpu) - np.asarray(xi_or)).max())


def tiny_workload(seed=0, huber_k=400.0, sigma_P=0.1):
    p = synth.tiny_pair(seed)
    cam = p["cam"]
    kw = dict(init_inv_depth=0.3, huber_k=huber_k, sigma_P=sigma_P)
    return dict(cam=cam, I_s=p["I_s"], N_s=p["normals_s"], frames=[p["I_t"]], iters=50, kw=kw)


def sequence_workload(name: str, n_frames: int, first: int = 1):
    cfg = SEQUENCE_CONFIGS[name]
    scene, cam = make_sequence_scene(cfg)
    poses = sequence_poses(cfg)
    I0, D0, N0, _ = render_sequence_frame(cfg, scene, cam, poses, 0, keyframe=True)
    frames = [render_sequence_frame(cfg, scene, cam, poses, f)[0] for f in range(first, first + n_frames)]
    iters = {"ppa256": 20, "vga": 20, "diff320": 30}[name]
    return dict(cam=cam, I_s=I0, N_s=N0, frames=frames, iters=iters, kw=dict(SEQ_PARAMS[name]),
                depth0=D0, poses=poses)


def K_of(cam):
    return (cam.fx, cam.fy, cam.cx, cam.cy)


def make_oracle(w, topology: int = 0, store_fp32: int = 0) -> "oracle.Oracle":
    o = oracle.Oracle(oracle.config_for_camera(w["cam"], topology=topology, store_fp32=store_fp32, **w["kw"]))
    o.set_keyframe(w["I_s"], w["N_s"])
    return o


def make_tracker(w, schedule=0, topology: int = 0):
    import paper_2606_03989_amd as pv
    cam = w["cam"]
    t = pv.Tracker(cam.H, cam.W, K_of(cam), **w["kw"])
    t.set_schedule(schedule)
    if topology:
        t.set_topology(topology)
    t.set_keyframe(w["I_s"], w["N_s"])
    return t


def diff_crop_workload(size: int = 24, n_frames: int = 2, seed: int = 3):
    """Centred size x size crop of the 320x240 differentiation sequence
    (intrinsics shifted by the crop origin), a perturbed sigma_D map around
    the sequence's 5e-3 and random output cotangents."""
    w = sequence_workload("diff320", n_frames)
    cam = w["cam"]
    x0, y0 = (cam.W - size) // 2, (cam.H - size) // 2
    crop = lambda a: np.ascontiguousarray(a[y0:y0 + size, x0:x0 + size])
    ccam = synth.Camera(H=size, W=size, fx=cam.fx, fy=cam.fy, cx=cam.cx - x0, cy=cam.cy - y0)
    rng = np.random.default_rng(seed)
    sig = (5e-3 * (1.0 + 0.2 * rng.uniform(-1.0, 1.0, (size, size)))).astype(np.float32)
    cxi = rng.normal(size=(n_frames, 6))
    crho = (rng.normal(size=(n_frames, size, size)) / (size * size)).astype(np.float32)
    return dict(cam=ccam, I_s=crop(w["I_s"]), N_s=crop(w["N_s"]), frames=[crop(f) for f in w["frames"]],
                sigma_map=sig, sigma_N=float(np.float32(1e-3)), huber_k=10.0, kw=dict(sigma_P=0.01), cxi=cxi, crho=crho)


def diff_full_workload(n_frames: int = 1, seed: int = 4):
    """The full 320x240 differentiation sequence with a perturbed sigma map."""
    w = sequence_workload("diff320", n_frames)
    cam = w["cam"]
    rng = np.random.default_rng(seed)
    sig = (5e-3 * (1.0 + 0.2 * rng.uniform(-1.0, 1.0, (cam.H, cam.W)))).astype(np.float32)
    cxi = rng.normal(size=(n_frames, 6))
    crho = (rng.normal(size=(n_frames, cam.H, cam.W)) / (cam.H * cam.W)).astype(np.float32)
    return dict(cam=cam, I_s=w["I_s"], N_s=w["N_s"], frames=w["frames"], sigma_map=sig, sigma_N=float(np.float32(1e-3)),
                huber_k=10.0, kw=dict(sigma_P=0.01), cxi=cxi, crho=crho)


def make_unroll(w, n_iters: int, ckpt_every: int):
    import paper_2606_03989_amd as pv
    cam = w["cam"]
    u = pv.Unrolled(cam.H, cam.W, K_of(cam), n_iters=n_iters, max_frames=len(w["frames"]),
                    ckpt_every=ckpt_every, **w["kw"])
    u.set_keyframe(w["I_s"], w["N_s"])
    return u


def make_unrolled_oracle(w, n_iters: int):
    from oracle.gradient import UnrolledOracle
    return UnrolledOracle(w["cam"], w["I_s"], w["N_s"], w["frames"], n_iters, w["sigma_map"], w["sigma_N"],
                          w["huber_k"], **w["kw"])


def noisy_sequence_workload(name: str, n_frames: int, theta):
    """A sequence workload whose keyframe and target frames go through the
    sensor-noise model instead of the sequence's Gaussian pixel noise."""
    from synth.noise import render_noisy_frame
    cfg = SEQUENCE_CONFIGS[name]
    scene, cam = make_sequence_scene(cfg)
    poses = sequence_poses(cfg)
    I0, D0, N0 = render_noisy_frame(cfg, scene, cam, poses, 0, theta, keyframe=True)
    frames = [render_noisy_frame(cfg, scene, cam, poses, f, theta)[0] for f in range(1, n_frames + 1)]
    iters = {"ppa256": 20, "vga": 20, "diff320": 30}[name]
    return dict(cam=cam, I_s=I0, N_s=N0, frames=frames, iters=iters, kw=dict(SEQ_PARAMS[name]), depth0=D0,
                poses=poses)


# --- the oracle's own sensitivity -------------------------------------------------

FP32_REL = 6e-8      # half an FP32 ulp, relative


def _max_agreement(items):
    """Element-wise maximum over (pose, depth-agreement) pairs; the depth
    dicts also carry the valid-fraction difference ("valid")."""
    pose = max(p for p, _ in items)
    depth = {k: max(d[k] for _, d in items) for k in ("rms", "p99", "max", "valid")}
    return pose, depth


def oracle_spread(w, frame, n_iters, start=None, topology: int = 0, ref=None, setup=None):
    """How far the oracle's own free-running result moves at the GPU's storage
    precision: (pose, depth-agreement dict), the element-wise maximum over two
    exact runs whose starting log-depths move by up to FP32_REL relative
    (seeded) and runs of the oracle's FP32 storage emulation, one from the same
    start and the others from moved starts (seven below 100k pixels, where runs
    are cheap and the spread of a sensitive horizon is a wide distribution,
    three above). `start`: the FP64 starting state (the oracle's exchange
    layout), else the keyframe reset state; `ref`: the unperturbed exact run's
    track output; `setup(oracle)` reproduces run-time settings on each fresh
    oracle."""
    tree = topology != 0

    def fresh(store):
        o = make_oracle(w, topology, store_fp32=store)
        if setup is not None:
            setup(o)
        if start is not None:
            o.set_state(start)
        return o

    if ref is None:
        o = fresh(0)
        ref = o.track(frame, n_iters)
        o.close()
    out = []
    n_pix = w["cam"].H * w["cam"].W
    store_seeds = (None, 2, 3, 4, 5, 6, 7, 8) if n_pix <= 100_000 else (None, 2, 3, 4)
    for store, seed in ((0, 0), (0, 1)) + tuple((1, sd) for sd in store_seeds):
        o = fresh(store)
        if seed is not None:
            st = o.get_state()
            pix = st[0] if tree else st
            rng = np.random.default_rng(seed)
            pix[..., 6] *= 1.0 + FP32_REL * rng.uniform(-1.0, 1.0, pix[..., 6].shape)
            o.set_state(st)
        r = o.track(frame, n_iters)
        da = depth_agreement(r["inv_depth"], ref["inv_depth"])
        da["valid"] = abs(r["valid_fraction"] - ref["valid_fraction"])
        out.append((pose_agreement(ref["xi"], r["xi"]), da))
        o.close()
    return _max_agreement(out)


VALID_TOL = 2e-3      # valid-warp fraction


def free_running_bounds(spread):
    """Bounds of a free-running comparison: the fixed bar or twice the
    oracle's own spread, whichever is larger (pose, depth RMS / p99 / max,
    valid-warp fraction)."""
    sp, sd = spread
    b = {k: max(DEPTH_TOL, 2.0 * sd[k]) for k in ("rms", "p99", "max")}
    b["valid"] = max(VALID_TOL, 2.0 * sd.get("valid", 0.0))
    return max(POSE_TOL, 2.0 * sp), b


def check_free_running(rg, ro, spread, name):
    """Asserts a free-running comparison against free_running_bounds; prints
    the measured agreement, the spread and the bounds."""
    dp = pose_agreement(rg["xi"], ro["xi"])
    da = depth_agreement(rg["inv_depth"], ro["inv_depth"])
    bp, bd = free_running_bounds(spread)
    sp, sd = spread
    print(f"{name}: pose {dp:.2e} (bound {bp:.2e}); depth rms {da['rms']:.2e} p99 {da['p99']:.2e} "
          f"max {da['max']:.2e} (bounds {bd['rms']:.2e} {bd['p99']:.2e} {bd['max']:.2e}); oracle spread "
          f"pose {sp:.2e} rms {sd['rms']:.2e} p99 {sd['p99']:.2e} max {sd['max']:.2e} "
          f"valid {sd.get('valid', 0.0):.2e}; valid {rg['valid_fraction']:.4f}/{ro['valid_fraction']:.4f}",
          flush=True)
    assert dp <= bp, f"{name}: pose {dp:.2e} > {bp:.2e}"
    for k in ("rms", "p99", "max"):
        assert da[k] <= bd[k], f"{name}: depth {k} {da[k]:.2e} > {bd[k]:.2e}"
    dv = abs(rg["valid_fraction"] - ro["valid_fraction"])
    assert dv <= bd["valid"], f"{name}: valid fraction differs by {dv:.2e} > {bd['valid']:.2e}"
    assert (rg["flags"] & oracle.DIVERGED) == (ro["flags"] & oracle.DIVERGED)
    return dp, da


def plane_errors(g, r):
    """Element-wise error of (planes, ...) arrays relative to each plane's
    largest magnitude in r."""
    g = np.asarray(g, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    n = r.shape[0]
    scale = np.abs(r).reshape(n, -1).max(axis=1).reshape((n,) + (1,) * (r.ndim - 1)) + 1e-30
    return np.abs(g - r) / scale


def iteration_spread(w, s32, frame, topology: int = 0, setup=None):
    """The oracle's own change, in plane-relative error, of one iteration from
    the FP32 state s32 at the GPU's storage precision: two exact runs from
    s32 with every element moved by up to FP32_REL relative (seeded), and four
    runs of the oracle's FP32 storage emulation (new messages rounded before
    the update), from s32 and from three moved copies of s32. Returns dict(plane_max=per-plane
    maximum, p999=99.9th percentile over all elements); for the quadtree one
    such dict per part ("pixels", "nodes"). `setup(oracle)` reproduces run-time
    settings (prior means) on each fresh oracle."""
    tree = topology != 0

    def one(state64, store):
        o = make_oracle(w, topology, store_fp32=store)
        if setup is not None:
            setup(o)
        o.set_state(state64)
        o.set_frame(frame)
        o.iterate(1)
        st = o.get_state()
        o.close()
        if tree:
            return tree_from_oracle(st)
        return from_oracle(st)

    def moved(seed):
        rng = np.random.default_rng(seed)
        if tree:
            return tree_to_oracle(tuple(a.astype(np.float64) * (1.0 + FP32_REL * rng.uniform(-1.0, 1.0, a.shape))
                                        for a in s32))
        return to_oracle(s32.astype(np.float64) * (1.0 + FP32_REL * rng.uniform(-1.0, 1.0, s32.shape)))

    def fold(acc, a, b):
        e = plane_errors(a, b)
        pm = e.reshape(e.shape[0], -1).max(axis=1)
        q = float(np.percentile(e, 99.9))
        if acc is None:
            return dict(plane_max=pm, p999=q)
        return dict(plane_max=np.maximum(acc["plane_max"], pm), p999=max(acc["p999"], q))

    exact = tree_to_oracle(s32) if tree else to_oracle(s32)
    base = one(exact, 0)
    runs = [one(moved(0), 0), one(moved(1), 0), one(exact, 1)] + [one(moved(sd), 1) for sd in (2, 3, 4)]
    if tree:
        res = {"pixels": None, "nodes": None}
        for r in runs:
            res["pixels"] = fold(res["pixels"], r[0], base[0])
            res["nodes"] = fold(res["nodes"], r[1], base[1])
        return res
    res = None
    for r in runs:
        res = fold(res, r, base)
    return res


SINGLE_BAR = 1e-5


def check_iteration(err, spread, name):
    """Bounds one teacher-forced iteration's plane-relative errors: each
    plane's maximum within SINGLE_BAR or twice the oracle's own spread of that
    plane, and the 99.9th percentile over all elements within SINGLE_BAR or
    twice the spread's. spread None: the fixed bar."""
    n = err.shape[0]
    pm = err.reshape(n, -1).max(axis=1)
    q = float(np.percentile(err, 99.9))
    if spread is None:
        bmax = np.full(n, SINGLE_BAR)
        bq = SINGLE_BAR
    else:
        bmax = np.maximum(SINGLE_BAR, 2.0 * spread["plane_max"])
        bq = max(SINGLE_BAR, 2.0 * spread["p999"])
    worst = np.unravel_index(np.argmax(err), err.shape)
    ratio = pm / bmax
    k = int(np.argmax(ratio))
    print(f"{name}: max {err.max():.2e} at {tuple(int(i) for i in worst)}, p99.9 {q:.2e} (bound {bq:.2e}); "
          f"tightest plane {k}: max {pm[k]:.2e} of bound {bmax[k]:.2e}", flush=True)
    bad = np.nonzero(pm > bmax)[0]
    assert bad.size == 0, f"{name}: planes {bad.tolist()[:8]} exceed their bounds ({pm[bad][:4]} > {bmax[bad][:4]})"
    assert q <= bq, f"{name}: p99.9 {q:.2e} > {bq:.2e}"
    return float(err.max()), q
