"""Benchmark of the per-pixel GBP hot path on one MI355X.

A step tracks one 640x480 frame of the seeded piecewise-planar sequence
(12 planes, inverse depths U[0.2, 2.0], pixel noise 0.02, 10% occluders):
frame preparation, 20 synchronous GBP iterations (fused schedule), pose and
statistics reductions and the inverse-depth/variance maps, re-anchoring when
the keyframe test fires. Frames are staged in device memory before timing.

Prints one JSON line: throughput in Mpixel-iter/s, the roofline of the
dominant kernel (the fused iteration pass, timed with HIP events on the
library stream), the FP64 CPU oracle timed on a bounded sample of the same
workload, and the per-factor schedule measured on the same GPU.

  python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
# algorithmic bytes per pixel-iteration of one fused pass: the 123 FP32 state
# values read and written once, the keyframe intensity and two normal targets,
# and one read of the warped target intensity and its two gradients
STATE_PLANES = 123
BYTES_PER_PX_ITER = STATE_PLANES * 4 * 2 + 4 + 8 + 12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fused_iterate_vga.json")
KERNEL_SOURCES = ["paper_2606_03989_amd/csrc/gbp_kernels.hip", "paper_2606_03989_amd/csrc/gbp_device.hpp"]
TREE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_quadtree_iterate_vga.json")
TREE_KERNEL_SOURCES = ["paper_2606_03989_amd/csrc/gbp_tree.hip", "paper_2606_03989_amd/csrc/gbp_tree.h",
                       "paper_2606_03989_amd/csrc/gbp_device.hpp"]


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def vga_inputs(n_frames: int):
    import numpy as np
    from synth.scenes import SEQUENCE_CONFIGS, make_sequence_scene, render_sequence_frame, sequence_poses
    cfg = SEQUENCE_CONFIGS["vga"]
    scene, cam = make_sequence_scene(cfg)
    poses = sequence_poses(cfg)
    I0, _, N0, _ = render_sequence_frame(cfg, scene, cam, poses, 0, keyframe=True)
    frames, normals = [], []
    for f in range(1, n_frames + 1):
        img, _, nrm, _ = render_sequence_frame(cfg, scene, cam, poses, f % cfg.n_frames)
        frames.append(img)
        normals.append(np.ascontiguousarray(nrm))
    return cam, I0, np.ascontiguousarray(N0), frames, normals


VGA_PARAMS = dict(sigma_P=0.01, huber_k=10.0)


def run_gpu(args):
    import numpy as np
    import torch
    import paper_2606_03989_amd as pv

    n_frames = args.warmup + args.steps
    log(f"rendering {n_frames} frames of the 640x480 sequence")
    cam, I0, N0, frames, normals = vga_inputs(n_frames)
    H, W = cam.H, cam.W
    dev = torch.device("cuda:0")
    d_I0 = torch.from_numpy(I0).to(dev)
    d_N0 = torch.from_numpy(N0).to(dev)
    d_frames = [torch.from_numpy(f).to(dev) for f in frames]
    d_normals = [torch.from_numpy(n).to(dev) for n in normals]
    stream = torch.cuda.current_stream()

    def make(schedule):
        t = pv.Tracker(H, W, (cam.fx, cam.fy, cam.cx, cam.cy), **VGA_PARAMS)
        t.set_stream(stream)
        t.set_schedule(schedule)
        t.set_keyframe(d_I0, d_N0)
        return t

    def step(t, i, iters):
        r = t.track(d_frames[i], iters, maps=True, out_device=True)
        if r["flags"] & pv.KEYFRAME_DUE:
            t.set_keyframe(d_frames[i], d_normals[i])
        return r

    iters = args.iters
    t = make(pv.SCHED_FUSED)
    for i in range(args.warmup):
        step(t, i, iters)
    torch.cuda.synchronize()
    t.profile(True)
    for k in range(4):
        t.profile_read(k)
    t0 = time.perf_counter()
    flags = 0
    for i in range(args.warmup, args.warmup + args.steps):
        r = step(t, i, iters)
        flags |= r["flags"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    it_ms, it_n = t.profile_read(pv.PROF_FUSED_ITERATE)
    fin_ms, fin_n = t.profile_read(pv.PROF_FUSED_FINAL)
    pro_ms, pro_n = t.profile_read(pv.PROF_FUSED_PROLOGUE)
    t.profile(False)
    elapsed = t1 - t0
    px_iters = H * W * iters * args.steps
    value = px_iters / elapsed / 1e6
    log(f"fused: {elapsed * 1e3 / args.steps:.3f} ms/step, {value:.1f} Mpx-iter/s; "
        f"iterate pass {it_ms / max(it_n, 1) * 1e3:.1f} us x {it_n}, final {fin_ms / max(fin_n, 1) * 1e3:.1f} us, "
        f"prologue {pro_ms / max(pro_n, 1) * 1e3:.1f} us; flags seen {flags}")

    avg_launch_s = it_ms / 1e3 / max(it_n, 1)
    bytes_per_launch = BYTES_PER_PX_ITER * H * W
    achieved = bytes_per_launch / avg_launch_s / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_source_hash") == kernel_source_hash():
            traffic = tr.get("bytes_per_launch")
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    kernel="k_fu_iterate<false>", bytes_per_px_iter=BYTES_PER_PX_ITER,
                    avg_launch_us=round(avg_launch_s * 1e6, 2), launches=it_n)

    # the frame step replayed as one graph against the same passes launched one
    # by one, both without profiling events, on the same frames
    def timed_steps(graph):
        tt = make(pv.SCHED_FUSED)
        tt.set_graph(graph)
        for i in range(args.warmup):
            step(tt, i, iters)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for i in range(args.warmup, args.warmup + args.steps):
            step(tt, i, iters)
        torch.cuda.synchronize()
        dt = time.perf_counter() - a
        tt.close()
        return dt * 1e3 / args.steps

    g_ms, u_ms = timed_steps(True), timed_steps(False)
    passes_ms = (it_ms + fin_ms + pro_ms) / args.steps
    frame_step = dict(graph_ms=round(g_ms, 3), unrolled_ms=round(u_ms, 3), passes_ms=round(passes_ms, 3),
                      overhead_graph_us=round((g_ms - passes_ms) * 1e3, 1),
                      overhead_unrolled_us=round((u_ms - passes_ms) * 1e3, 1),
                      overhead_removed_us=round((u_ms - g_ms) * 1e3, 1))
    log(f"frame step: graph replay {g_ms:.3f} ms, passes launched one by one {u_ms:.3f} ms, "
        f"prologue + passes {passes_ms:.3f} ms: {(u_ms - g_ms) * 1e3:.1f} us per frame removed by the graph")

    # the per-factor schedule on the same frames (the schedule comparison's baseline)
    per_factor = None
    if args.per_factor_steps > 0:
        tp = make(pv.SCHED_PER_FACTOR)
        for i in range(min(args.warmup, 1)):
            step(tp, i, iters)
        torch.cuda.synchronize()
        tp.profile(True)
        tp.profile_read(pv.PROF_PER_FACTOR)
        a = time.perf_counter()
        ns = min(args.per_factor_steps, args.steps)
        for i in range(args.warmup, args.warmup + ns):
            step(tp, i, iters)
        torch.cuda.synchronize()
        b = time.perf_counter()
        pf_ms, pf_n = tp.profile_read(pv.PROF_PER_FACTOR)
        pf_value = H * W * iters * ns / (b - a) / 1e6
        pf_launch = pf_ms / 1e3 / max(pf_n, 1)
        per_factor = dict(value=round(pf_value, 1), unit="Mpixel-iter/s", steps=ns,
                          iteration_us=round(pf_launch * 1e6, 1),
                          frac_of_fused_bytes=round(BYTES_PER_PX_ITER * H * W / pf_launch / 1e9 / HBM_PEAK_GBS, 4),
                          fused_speedup=round(value / pf_value, 2))
        log(f"per-factor: {pf_value:.1f} Mpx-iter/s, iteration {pf_launch * 1e6:.1f} us")
        tp.close()
    t.close()
    return dict(value=value, elapsed=elapsed, roofline=roofline, per_factor=per_factor, frame_step=frame_step,
                H=H, W=W, iters=iters,
                pass_us=avg_launch_s * 1e6, inputs=(cam, d_I0, d_N0, d_frames, d_normals, stream))


# algorithmic bytes of one quadtree iteration (pixel pass + node pass).
# Pixel: reads its point (7), normal slots (8), the parent's partial for its
# slot (27), a quarter of the parent's pose (1.5), keyframe intensity and two
# normal targets (3), the warped target intensity and gradients (3); writes
# its point (7), its partial to the parent (27), four normal partials (8).
# Node: reads its pose (6), a quarter of the parent's pose (1.5), the parent's
# partial (27), four children's poses (24) and partials (108); writes its pose
# (6), its partial to the parent (27) and four partials to the children (108).
TREE_PIXEL_FLOATS = 49.5 + 42
TREE_NODE_FLOATS = 166.5 + 141


def run_quadtree(args, g):
    """The same frames with the quadtree identity topology (Fig. 2): per-pass
    duration (pixel and node launches together) against the grid's pass."""
    import torch
    import paper_2606_03989_amd as pv
    cam, d_I0, d_N0, d_frames, d_normals, stream = g["inputs"]
    H, W, iters = g["H"], g["W"], g["iters"]
    t = pv.Tracker(H, W, (cam.fx, cam.fy, cam.cx, cam.cy), **VGA_PARAMS)
    t.set_stream(stream)
    t.set_topology(pv.TOPO_QUADTREE)
    t.set_keyframe(d_I0, d_N0)
    n_nodes = sum(h * w for h, w in t.tree_levels()[1:])
    levels = len(t.tree_levels())

    def step(i):
        r = t.track(d_frames[i], iters, maps=True, out_device=True)
        if r["flags"] & pv.KEYFRAME_DUE:
            t.set_keyframe(d_frames[i], d_normals[i])
        return r

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t.profile(True)
    for k in range(4):
        t.profile_read(k)
    a = time.perf_counter()
    flags = 0
    for i in range(args.warmup, args.warmup + args.steps):
        flags |= step(i)["flags"]
    torch.cuda.synchronize()
    b = time.perf_counter()
    it_ms, it_n = t.profile_read(pv.PROF_FUSED_ITERATE)
    t.profile(False)
    t.close()
    value = H * W * iters * args.steps / (b - a) / 1e6
    pass_s = it_ms / 1e3 / max(it_n, 1)
    bytes_per_pass = 4.0 * (TREE_PIXEL_FLOATS * H * W + TREE_NODE_FLOATS * n_nodes)
    achieved = bytes_per_pass / pass_s / 1e9
    log(f"quadtree: {value:.1f} Mpx-iter/s, pass {pass_s * 1e6:.1f} us ({levels} levels, {n_nodes} nodes), "
        f"{achieved:.0f} GB/s algorithmic; flags seen {flags}")
    traffic = None
    if os.path.exists(TREE_TRAFFIC_FILE):
        with open(TREE_TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_source_hash") == kernel_source_hash(TREE_KERNEL_SOURCES):
            traffic = tr.get("bytes_per_pass")
    return dict(value=round(value, 1), unit="Mpixel-iter/s", levels=levels, nodes=n_nodes,
                pass_us=round(pass_s * 1e6, 2), grid_pass_us=round(g["pass_us"], 2),
                pass_speedup_vs_grid=round(g["pass_us"] / (pass_s * 1e6), 3),
                bytes_per_pass=int(bytes_per_pass), traffic=traffic, achieved_GBs=round(achieved, 1),
                frac=round(achieved / HBM_PEAK_GBS, 4), vs_grid=round(value / g["value"], 3))


def _render_seq(args):
    s, n_frames = args
    import numpy as np
    from synth.scenes import batch_sequence_config, make_sequence_scene, render_sequence_frame, sequence_poses
    cfg = batch_sequence_config(s)
    scene, cam = make_sequence_scene(cfg)
    poses = sequence_poses(cfg)
    I0, _, N0, _ = render_sequence_frame(cfg, scene, cam, poses, 0, keyframe=True)
    frames = [render_sequence_frame(cfg, scene, cam, poses, f)[0] for f in range(1, n_frames + 1)]
    return cam, I0, np.ascontiguousarray(N0), frames


# anonymous shared mappings (one per sequence) that the forked render workers
# fill: frames 1..n, then their normal maps
_SHARED = {}


def _render_seq_shared(args):
    """Renders sequence s's keyframe and target frames 1..n_frames with their
    normal maps into the anonymous shared mapping _SHARED[s] (created by the
    parent before the workers fork); returns the keyframe."""
    s, n_frames = args
    import numpy as np
    from synth.scenes import batch_sequence_config, make_sequence_scene, render_sequence_frame, sequence_poses
    cfg = batch_sequence_config(s)
    scene, cam = make_sequence_scene(cfg)
    poses = sequence_poses(cfg)
    I0, _, N0, _ = render_sequence_frame(cfg, scene, cam, poses, 0, keyframe=True)
    buf = _SHARED[s]
    n = cam.H * cam.W
    fr = np.ndarray((n_frames, cam.H, cam.W), np.float32, buffer=buf, offset=0)
    nm = np.ndarray((n_frames, cam.H, cam.W, 3), np.float32, buffer=buf, offset=4 * n_frames * n)
    for f in range(n_frames):
        img, _, nrm, _ = render_sequence_frame(cfg, scene, cam, poses, f + 1)
        fr[f] = img
        nm[f] = nrm
    del fr, nm
    return cam, I0, np.ascontiguousarray(N0, dtype=np.float32)


BATCH_PARAMS = dict(sigma_P=0.01, huber_k=400.0)


def run_batch(n_seq: int, n_frames: int, iters: int, plain_steps: int, persistent_steps: int = 8,
              kf_frames: int = 16):
    """64 seeded 50-frame sequences, resolutions cycling 128x96, 256x256,
    320x240, 640x480; frames 1..n_frames are tracked after keyframe 0; each
    step advances every sequence by one distinct frame
    (`iters` iterations) with the keyframe test and re-anchoring on the device
    inside the step. Frames 1 and 2 warm up (graph capture, tile autotuning);
    frames 3..n_frames are timed. The batch runs one launch per pass over all
    sequences in a graph-captured frame step; the persistent variant (one
    cooperative launch per iteration block) is timed on frames 3.. in a second
    batch; the plain leg runs the same sequences one after another in
    per-sequence contexts. Keyframes are re-anchored every `kf_frames`
    frames (the paper's 150 exceeds a 50-frame sequence), so the timed steps
    include the device-side re-anchoring."""
    import mmap
    import multiprocessing as mp
    import numpy as np
    import torch
    import paper_2606_03989_amd as pv
    from synth.scenes import batch_resolution
    from synth.scenes import batch_sequence_config
    dev = torch.device("cuda:0")
    n_max = batch_sequence_config(0).n_frames - 1
    if not 2 < n_frames <= n_max:
        raise SystemExit(f"--batch-frames must be in 3..{n_max} (frames after the keyframe)")
    shapes = [batch_resolution(s) for s in range(n_seq)]
    for s, (H, W) in enumerate(shapes):
        _SHARED[s] = mmap.mmap(-1, 16 * n_frames * H * W)
    try:
        with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
            data = pool.map(_render_seq_shared, [(s, n_frames) for s in range(n_seq)])
        fr, nm = [], []
        for s, (H, W) in enumerate(shapes):
            a = np.ndarray((n_frames, H, W), np.float32, buffer=_SHARED[s], offset=0)
            b_ = np.ndarray((n_frames, H, W, 3), np.float32, buffer=_SHARED[s], offset=4 * n_frames * H * W)
            fr.append([f for f in torch.from_numpy(a.copy()).to(dev)])
            nm.append([x for x in torch.from_numpy(b_.copy()).to(dev)])
            del a, b_
    finally:
        for s in list(_SHARED):
            _SHARED.pop(s).close()
    cams = [d[0] for d in data]
    Ks = [(c.fx, c.fy, c.cx, c.cy) for c in cams]
    kf = [torch.from_numpy(d[1]).to(dev) for d in data]
    kn = [torch.from_numpy(d[2]).to(dev) for d in data]
    px = sum(h * w for h, w in shapes)
    stream = torch.cuda.current_stream()

    def make(persistent):
        b = pv.Batch(shapes, Ks, kf_max_frames=kf_frames, **BATCH_PARAMS)
        b.set_stream(stream)
        b.set_persistent(persistent)
        b.set_keyframes(list(range(n_seq)), kf, kn)
        return b

    def step(b, f):
        return b.track([x[f] for x in fr], iters, normals=[x[f] for x in nm])

    b = make(False)
    step(b, 0)                                         # warm-up, graph capture
    tx, ty = b.autotune(iters)
    step(b, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ms, flags, reanchored = [], 0, 0
    for f in range(2, n_frames):
        r = step(b, f)
        step_ms.append(b.last_step_ms())
        for o in r:
            flags |= o["flags"]
            reanchored += 1 if o["flags"] & pv.KEYFRAME_DUE else 0
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    steps = n_frames - 2
    batch_value = px * iters * steps / tb / 1e6
    b.close()
    log(f"batched: {n_seq} sequences, {px} px, frames 3-{n_frames}, tile {tx}x{ty}: {tb * 1e3 / steps:.2f} ms/step "
        f"(graph {sum(step_ms) / len(step_ms):.2f} ms) -> {batch_value:.1f} Mpx-iter/s; flags seen {flags}, "
        f"{reanchored} re-anchorings")

    persistent = None
    if persistent_steps > 0:
        bp = make(True)
        bp.set_tile(tx, ty)
        step(bp, 0)
        step(bp, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ns = min(persistent_steps, n_frames - 2)
        pms = []
        for f in range(2, 2 + ns):
            step(bp, f)
            pms.append(bp.last_step_ms())
        torch.cuda.synchronize()
        tpp = time.perf_counter() - t0
        bp.close()
        persistent = dict(value=round(px * iters * ns / tpp / 1e6, 1), ms_per_step=round(tpp * 1e3 / ns, 3),
                          step_event_ms=round(sum(pms) / len(pms), 3), steps=ns,
                          launch_per_pass_step_event_ms=round(sum(step_ms[:ns]) / ns, 3))
        log(f"batched, persistent iteration block: {tpp * 1e3 / ns:.2f} ms/step (events {sum(pms) / len(pms):.2f} ms) "
            f"against {sum(step_ms[:ns]) / ns:.2f} ms with one launch per pass on the same frames")

    plain = []
    for s in range(n_seq):
        t = pv.Tracker(shapes[s][0], shapes[s][1], Ks[s], **BATCH_PARAMS)
        t.set_stream(stream)
        t.set_keyframe(kf[s], kn[s])
        t.track(fr[s][0], iters, maps=False)
        plain.append(t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(plain_steps):
        for s in range(n_seq):
            plain[s].track(fr[s][1 + k], iters, maps=False)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    plain_value = px * iters * plain_steps / tp / 1e6
    for t in plain:
        t.close()
    log(f"plain per-sequence contexts: {tp * 1e3 / plain_steps:.2f} ms/step -> {plain_value:.1f} Mpx-iter/s")
    return dict(value=round(batch_value, 1), unit="Mpixel-iter/s", sequences=n_seq, pixels=px, iters_per_frame=iters,
                frames_per_sequence=n_frames + 1, tracked_frames=n_frames, steps=steps, ms_per_step=round(tb * 1e3 / steps, 3), tile=[tx, ty],
                flags_seen=flags, reanchorings=reanchored, persistent=persistent,
                plain_value=round(plain_value, 1), plain_ms_per_step=round(tp * 1e3 / plain_steps, 3),
                speedup_vs_plain=round(batch_value / plain_value, 3),
                resolutions="128x96, 256x256, 320x240, 640x480 (16 each)",
                reanchoring="keyframe test and re-anchoring on the device inside each captured frame step",
                kf_max_frames=kf_frames)


DIFF_PARAMS = dict(sigma_P=0.01, huber_k=10.0)


def run_adjoint(n_frames: int, iters: int, ckpt: int, reps: int):
    """Forward + adjoint over the 320x240 differentiation sequence: n_frames
    frames of `iters` unrolled iterations with a checkpoint every `ckpt`, the
    adjoint for output cotangents of the pose and inverse-depth outputs
    (random, seeded), against the plain fused forward on the same frames."""
    import numpy as np
    import torch
    import paper_2606_03989_amd as pv
    from synth.scenes import SEQUENCE_CONFIGS, make_sequence_scene, render_sequence_frame, sequence_poses
    cfg = SEQUENCE_CONFIGS["diff320"]
    scene, cam = make_sequence_scene(cfg)
    poses = sequence_poses(cfg)
    I0, _, N0, _ = render_sequence_frame(cfg, scene, cam, poses, 0, keyframe=True)
    frames = np.stack([render_sequence_frame(cfg, scene, cam, poses, f)[0] for f in range(1, n_frames + 1)])
    H, W = cam.H, cam.W
    K = (cam.fx, cam.fy, cam.cx, cam.cy)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    d_fr = torch.from_numpy(frames.astype(np.float32)).to(dev)
    d_I0, d_N0 = torch.from_numpy(I0).to(dev), torch.from_numpy(np.ascontiguousarray(N0)).to(dev)
    sig = torch.full((H, W), 5e-3, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(11)
    cxi = rng.normal(size=(n_frames, 6))
    crho = torch.from_numpy((rng.normal(size=(n_frames, H, W)) / (H * W)).astype(np.float32)).to(dev)
    u = pv.Unrolled(H, W, K, n_iters=iters, max_frames=n_frames, ckpt_every=ckpt, **DIFF_PARAMS)
    u.set_stream(stream)
    u.set_keyframe(d_I0, d_N0)
    u.forward(d_fr, sig, 1e-3, DIFF_PARAMS["huber_k"], out_device=True)      # warm-up
    u.backward(cxi, crho, grad_device=True)
    torch.cuda.synchronize()
    tf = tb = 0.0
    for _ in range(reps):
        a = time.perf_counter()
        u.forward(d_fr, sig, 1e-3, DIFF_PARAMS["huber_k"], out_device=True)
        torch.cuda.synchronize()
        b = time.perf_counter()
        u.backward(cxi, crho, grad_device=True)
        torch.cuda.synchronize()
        c = time.perf_counter()
        tf += b - a
        tb += c - b
    fwd_ms, bwd_ms = u.last_ms()
    u.close()
    t = pv.Tracker(H, W, K, sigma_N=1e-3, **DIFF_PARAMS)
    t.set_stream(stream)
    t.set_sigma_map(sig)
    t.set_keyframe(d_I0, d_N0)
    for f in range(n_frames):
        t.track(d_fr[f], iters, maps=False)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(reps):
        t.set_keyframe(d_I0, d_N0)
        for f in range(n_frames):
            t.track(d_fr[f], iters, maps=False)
    torch.cuda.synchronize()
    tp = time.perf_counter() - a
    t.close()
    work = H * W * iters * n_frames * reps / 1e6
    v_fa = work / (tf + tb)
    v_plain = work / tp
    log(f"forward+adjoint: 320x240, {n_frames} frames x {iters} iterations, checkpoint every {ckpt}: "
        f"forward {tf * 1e3 / reps:.1f} ms, adjoint {tb * 1e3 / reps:.1f} ms -> {v_fa:.1f} Mpx-iter/s; "
        f"plain forward {tp * 1e3 / reps:.1f} ms -> {v_plain:.1f} Mpx-iter/s")
    return dict(value=round(v_fa, 2), unit="Mpixel-iter/s (forward px-iter / (forward with tape + adjoint))",
                workload=f"diff320 320x240, {n_frames} frames x {iters} unrolled iterations, checkpoint every {ckpt}",
                forward_ms=round(tf * 1e3 / reps, 3), adjoint_ms=round(tb * 1e3 / reps, 3),
                forward_event_ms=round(fwd_ms, 3), adjoint_event_ms=round(bwd_ms, 3),
                plain_forward_value=round(v_plain, 1), plain_forward_ms=round(tp * 1e3 / reps, 3),
                ratio_vs_plain=round(v_fa / v_plain, 4), gradients="sigma_D map, sigma_N, huber_k")


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(iters: int):
    """The FP64 oracle, as it stands, timed on the host's cores: all threads
    on the 32x24 pair in full (50 iterations), the 256x256 sequence's first 5
    frames (20 iterations each) and the 640x480 frame 1 (`iters` iterations);
    one thread on the 32x24 pair and 2 iterations of the 640x480 frame 1.
    `value` is the 640x480 sample on all threads (the metric's workload);
    about 15 s of CPU work on a 16-thread host."""
    import oracle
    from synth.scenes import SEQUENCE_CONFIGS, make_sequence_scene, render_sequence_frame, sequence_poses
    import synth

    def timed(cam, I0, N0, frames, n_it, kw):
        o = oracle.Oracle(oracle.config_for_camera(cam, **kw))
        o.set_keyframe(I0, N0)
        a = time.perf_counter()
        for f in frames:
            o.track(f, n_it)
        dt = time.perf_counter() - a
        o.close()
        return cam.H * cam.W * n_it * len(frames) / dt / 1e6, dt

    all_threads = oracle.threads()
    p = synth.tiny_pair(0)
    tiny = (p["cam"], p["I_s"], p["normals_s"], [p["I_t"]], 50, dict(init_inv_depth=0.3))
    cfg = SEQUENCE_CONFIGS["ppa256"]
    scene, cam2 = make_sequence_scene(cfg)
    poses = sequence_poses(cfg)
    I2, _, N2, _ = render_sequence_frame(cfg, scene, cam2, poses, 0, keyframe=True)
    fr2 = [render_sequence_frame(cfg, scene, cam2, poses, f)[0] for f in range(1, 6)]
    ppa = (cam2, I2, N2, fr2, 20, dict(sigma_P=0.01, huber_k=400.0))
    cam3, I3, N3, fr3, _ = vga_inputs(1)
    samples = {}
    for name, wl in (("tiny 32x24, 50 iterations", tiny), ("256x256, frames 1-5 x 20 iterations", ppa),
                     (f"640x480, frame 1 x {iters} iterations", (cam3, I3, N3, fr3, iters, VGA_PARAMS))):
        v, dt = timed(*wl)
        samples[name] = dict(Mpx_iter_s=round(v, 4), seconds=round(dt, 2), threads=all_threads)
        if name.startswith("640x480"):
            value, vdt = v, dt
    oracle.set_threads(1)
    try:
        for name, wl in (("tiny 32x24, 50 iterations", tiny),
                         ("640x480, frame 1 x 2 iterations", (cam3, I3, N3, fr3, 2, VGA_PARAMS))):
            v, dt = timed(*wl)
            samples[name + ", 1 thread"] = dict(Mpx_iter_s=round(v, 4), seconds=round(dt, 2), threads=1)
    finally:
        oracle.set_threads(all_threads)
    cpu = _cpu_model()
    log(f"oracle on {all_threads} threads of {cpu}: " +
        "; ".join(f"{k}: {d['Mpx_iter_s']} Mpx-iter/s ({d['seconds']} s)" for k, d in samples.items()))
    return dict(value=round(value, 4), unit="Mpixel-iter/s", cores=all_threads, kind="oracle",
                sample=f"frame 1 of the 640x480 sequence, {iters} GBP iterations ({vdt:.1f} s), all threads",
                cpu_model=cpu, samples=samples)


def noise_sweep(n_frames: int = 20, iters: int = 20):
    """Robustness of tracking to pixel-processor-array sensor noise (App. D.1).
    The 256x256 scene of the sequence workload with slow motion (2 mm and
    0.1 deg per frame at most, sub-pixel per frame), rendered without noise,
    with Gaussian pixel noise 0.01, and through the Poisson-Gaussian model
    with the mild and strong settings. Prints one JSON line; per setting over
    the frames: the median rotation error of Eq. (rel_err) in degrees, the
    median relative pose error of Eq. (rel_err) (translation carries the scale
    the log-depth prior fixes, so it includes a scale bias shared by all
    settings), and the median deviation of the pose from the noise-free run
    relative to the ground-truth motion. The "+temporal" runs carry each frame's
    estimates forward as the next frame's prior means."""
    import dataclasses
    import math
    import numpy as np
    import paper_2606_03989_amd as pv
    from synth import PPA_MILD, PPA_STRONG
    from synth.noise import degrade
    from synth.scenes import SEQUENCE_CONFIGS, make_sequence_scene, render, sequence_poses
    cfg = dataclasses.replace(SEQUENCE_CONFIGS["ppa256"], max_step_t=0.002, max_step_r_deg=0.1, noise_sigma=0.0)
    scene, cam = make_sequence_scene(cfg)
    poses = sequence_poses(cfg)
    K = (cam.fx, cam.fy, cam.cx, cam.cy)
    clean = [render(scene, cam, poses[f]) for f in range(n_frames + 1)]
    N0 = np.ascontiguousarray(clean[0][2], np.float32)

    def so3_log(R):
        c = max(-1.0, min(1.0, 0.5 * (np.trace(R) - 1.0)))
        th = math.acos(c)
        v = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
        return 0.5 * v if th < 1e-8 else th / (2.0 * math.sin(th)) * v

    def images(setting):
        out = []
        for f in range(n_frames + 1):
            img = clean[f][0]
            rng = np.random.default_rng([cfg.seed, f, 11, len(setting)])
            if setting == "gaussian":
                img = img + rng.normal(0.0, 0.01, img.shape)
            elif setting in ("mild", "strong"):
                img = degrade(img, PPA_MILD if setting == "mild" else PPA_STRONG, rng)
            out.append(np.ascontiguousarray(img, np.float32))
        return out

    runs = {}
    for setting in ("clean", "gaussian", "mild", "strong", "clean+temporal", "strong+temporal"):
        imgs = images(setting.split("+")[0])
        temporal = setting.endswith("+temporal")
        t = pv.Tracker(cam.H, cam.W, K, sigma_P=0.01, huber_k=400.0)
        t.set_keyframe(imgs[0], N0)
        xs, flags = [], 0
        for f in range(1, n_frames + 1):
            r = t.track(imgs[f], iters, maps=False)
            flags |= r["flags"]
            xs.append(r["xi"])
            if temporal:
                # motion continuity and depth propagation (Sec. 3.3)
                t.set_prior_from_state()
        t.close()
        runs[setting] = (xs, flags)
    out = {}
    for setting, (xs, flags) in runs.items():
        rot, rel, dev = [], [], []
        for f, xi in enumerate(xs, start=1):
            T = np.linalg.inv(poses[f]) @ poses[0]
            E = pv_exp(xi)
            er = so3_log(E[:3, :3] @ T[:3, :3].T)
            et = E[:3, 3] - T[:3, 3]
            wg = so3_log(T[:3, :3])
            den = math.sqrt(float(wg @ wg + T[:3, 3] @ T[:3, 3]))
            rot.append(math.degrees(float(np.linalg.norm(er))))
            rel.append(math.sqrt(float(er @ er + et @ et)) / den)
            dev.append(float(np.linalg.norm(np.asarray(xi) - np.asarray(runs["clean"][0][f - 1]))) / den)
        out[setting] = dict(median_rot_err_deg=round(float(np.median(rot)), 5), last_rel_pose_err=round(rel[-1], 4),
                            median_rel_pose_err=round(float(np.median(rel)), 4),
                            median_dev_from_clean=round(float(np.median(dev)), 5), flags=int(flags))
        log(f"{setting}: {out[setting]}")
    print(json.dumps({"noise_sweep": out,
                      "workload": f"256x256 six-plane scene, slow motion, frames 1-{n_frames}, {iters} iterations"}))


def compare_solvers(n_frames: int = 10):
    """Centralised IRLS Gauss-Newton against distributed GBP (Sec. 4.4, Fig.
    centralized_vs_pixvod) on the same GPU: the 256x256 slow-motion scene of
    the noise sweep, frames 1..n, each solver warm-started frame to frame.
    Prints one JSON line with, per solver and per-frame iteration count, the
    median rotation error and relative pose error of Eq. (rel_err) and the
    GPU time per frame."""
    import dataclasses
    import math
    import numpy as np
    import paper_2606_03989_amd as pv
    from synth.scenes import SEQUENCE_CONFIGS, make_sequence_scene, render, sequence_poses
    cfg = dataclasses.replace(SEQUENCE_CONFIGS["ppa256"], max_step_t=0.002, max_step_r_deg=0.1, noise_sigma=0.0)
    scene, cam = make_sequence_scene(cfg)
    poses = sequence_poses(cfg)
    K = (cam.fx, cam.fy, cam.cx, cam.cy)
    clean = [render(scene, cam, poses[f]) for f in range(n_frames + 1)]
    imgs = [np.ascontiguousarray(c[0], np.float32) for c in clean]
    N0 = np.ascontiguousarray(clean[0][2], np.float32)

    def so3_log(R):
        c = max(-1.0, min(1.0, 0.5 * (np.trace(R) - 1.0)))
        th = math.acos(c)
        v = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
        return 0.5 * v if th < 1e-8 else th / (2.0 * math.sin(th)) * v

    def errors(xs):
        rot, rel = [], []
        for f, xi in enumerate(xs, start=1):
            T = np.linalg.inv(poses[f]) @ poses[0]
            E = pv_exp(xi)
            er = so3_log(E[:3, :3] @ T[:3, :3].T)
            et = E[:3, 3] - T[:3, 3]
            wg = so3_log(T[:3, :3])
            rot.append(math.degrees(float(np.linalg.norm(er))))
            rel.append(math.sqrt(float(er @ er + et @ et)) / math.sqrt(float(wg @ wg + T[:3, 3] @ T[:3, 3])))
        return round(float(np.median(rot)), 5), round(float(np.median(rel)), 4)

    out = {}
    params = dict(sigma_P=0.01, huber_k=400.0)
    for name, topo in (("gbp_grid", pv.TOPO_GRID), ("gbp_quadtree", pv.TOPO_QUADTREE)):
        for iters in (20, 100):
            t = pv.Tracker(cam.H, cam.W, K, **params)
            if topo:
                t.set_topology(topo)
            t.set_keyframe(imgs[0], N0)
            xs, ms = [], 0.0
            for f in range(1, n_frames + 1):
                a = time.perf_counter()
                xs.append(t.track(imgs[f], iters, maps=False)["xi"])
                ms += (time.perf_counter() - a) * 1e3
            t.close()
            rot, rel = errors(xs)
            out[f"{name}_{iters}it"] = dict(median_rot_err_deg=rot, median_rel_pose_err=rel,
                                            ms_per_frame=round(ms / n_frames, 3))
            log(f"{name} {iters} iterations/frame: {out[f'{name}_{iters}it']}")
    for iters in (1, 3, 10):
        c = pv.Central(cam.H, cam.W, K, max_cg=400, cg_tol=1e-8, **params)
        c.set_keyframe(imgs[0], N0)
        xs, ms, cg = [], 0.0, 0
        for f in range(1, n_frames + 1):
            r = c.track(imgs[f], iters, maps=False)
            xs.append(r["xi"])
            ms += c.last_ms()
            cg += r["cg_iters"]
        c.close()
        rot, rel = errors(xs)
        out[f"centralised_{iters}it"] = dict(median_rot_err_deg=rot, median_rel_pose_err=rel,
                                             ms_per_frame=round(ms / n_frames, 3),
                                             cg_iterations_per_frame=round(cg / n_frames, 1))
        log(f"centralised {iters} IRLS iterations/frame: {out[f'centralised_{iters}it']}")
    print(json.dumps({"solver_comparison": out, "workload": f"256x256 six-plane scene, slow motion, frames 1-{n_frames}, "
                      "sigma_P 0.01, Huber k 400; centralised CG tolerance 1e-8"}))


def transfer_check(every: int = 5, n_frames: int = 20, iters: int = 20):
    """Re-anchoring with and without keyframe depth transfer (depth propagation,
    Sec. 3.3) on the 256x256 slow-motion scene: a new keyframe every `every`
    frames; after each re-anchoring, the inverse-depth error of the carried
    state against the rendered depth of the new keyframe, before any iteration
    on it and after the next frame. Also the duration of the transfer at
    640x480. Prints one JSON line."""
    import dataclasses
    import numpy as np
    import torch
    import paper_2606_03989_amd as pv
    from synth.scenes import SEQUENCE_CONFIGS, make_sequence_scene, render, sequence_poses
    cfg = dataclasses.replace(SEQUENCE_CONFIGS["ppa256"], max_step_t=0.002, max_step_r_deg=0.1, noise_sigma=0.0)
    scene, cam = make_sequence_scene(cfg)
    poses = sequence_poses(cfg)
    K = (cam.fx, cam.fy, cam.cx, cam.cy)
    frames = [render(scene, cam, poses[f]) for f in range(n_frames + 1)]
    out = {}
    for transfer in (False, True):
        t = pv.Tracker(cam.H, cam.W, K, sigma_P=0.01, huber_k=400.0)
        t.set_keyframe(np.ascontiguousarray(frames[0][0], np.float32), np.ascontiguousarray(frames[0][2], np.float32))
        before, after = [], []
        pending = None
        for f in range(1, n_frames + 1):
            img = np.ascontiguousarray(frames[f][0], np.float32)
            r = t.track(img, iters)
            if pending is not None:
                after.append(float(np.median(np.abs(r["inv_depth"] - pending) / pending)))
                pending = None
            if f % every == 0 and f < n_frames:
                t.set_keyframe(img, np.ascontiguousarray(frames[f][2], np.float32), transfer_depth=transfer)
                st = t.get_state()
                rho_true = 1.0 / frames[f][1]
                rho = np.exp(-st[6].astype(np.float64))
                before.append(float(np.median(np.abs(rho - rho_true) / rho_true)))
                pending = rho_true
        t.close()
        key = "transfer" if transfer else "carry_over"
        out[key] = dict(median_inv_depth_err_at_reanchor=round(float(np.mean(before)), 4),
                        median_inv_depth_err_after_next_frame=round(float(np.mean(after)), 4))
        log(f"{key}: {out[key]}")
    # duration of one transfer at 640x480
    cam2, I0, N0, fr, nr = vga_inputs(2)
    dev = torch.device("cuda:0")
    t = pv.Tracker(cam2.H, cam2.W, (cam2.fx, cam2.fy, cam2.cx, cam2.cy), **VGA_PARAMS)
    t.set_keyframe(torch.from_numpy(I0).to(dev), torch.from_numpy(N0).to(dev))
    d0, n0 = torch.from_numpy(fr[0]).to(dev), torch.from_numpy(nr[0]).to(dev)
    t.track(d0, 5, maps=False)
    ms = []
    for _ in range(5):
        torch.cuda.synchronize()
        a = time.perf_counter()
        t.set_keyframe(d0, n0, transfer_depth=True)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - a) * 1e3)
        t.track(d0, 1, maps=False)
    t.close()
    out["reanchor_with_transfer_ms_640x480"] = round(float(np.median(ms)), 3)
    print(json.dumps({"depth_transfer": out, "workload": f"256x256 six-plane scene, slow motion, keyframe every {every} "
                      f"frames, frames 1-{n_frames}, {iters} iterations; timing at 640x480"}))


def pv_exp(xi):
    """Exp of Eq. (exp_err) as a 4x4 matrix (reporting only)."""
    import numpy as np
    w, rho = np.asarray(xi[:3], float), np.asarray(xi[3:], float)
    th = float(np.linalg.norm(w))
    Wm = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-8:
        A, B, C = 1.0, 0.5, 1.0 / 6.0
    else:
        A, B, C = np.sin(th) / th, (1 - np.cos(th)) / th ** 2, (th - np.sin(th)) / th ** 3
    T = np.eye(4)
    T[:3, :3] = np.eye(3) + A * Wm + B * Wm @ Wm
    T[:3, 3] = (np.eye(3) + B * Wm + C * Wm @ Wm) @ rho
    return T


def probe(frames: int = 3, copy_mb: int = 512):
    """Short run for hardware-counter collection: the fused schedule on a few
    frames, one per-factor frame, the quadtree, a short forward+adjoint on the
    320x240 differentiation sequence (2 frames x 10 iterations) and a plain
    device copy of known size that calibrates the byte counters."""
    import torch
    import paper_2606_03989_amd as pv
    cam, I0, N0, fr, _ = vga_inputs(frames)
    dev = torch.device("cuda:0")
    d_fr = [torch.from_numpy(f).to(dev) for f in fr]
    for sched in (pv.SCHED_FUSED, pv.SCHED_PER_FACTOR):
        t = pv.Tracker(cam.H, cam.W, (cam.fx, cam.fy, cam.cx, cam.cy), **VGA_PARAMS)
        t.set_stream(torch.cuda.current_stream())
        t.set_schedule(sched)
        t.set_keyframe(torch.from_numpy(I0).to(dev), torch.from_numpy(N0).to(dev))
        for f in (d_fr if sched == pv.SCHED_FUSED else d_fr[:1]):
            t.track(f, 20, maps=False)
        t.close()
    # the quadtree topology on the same frames
    t = pv.Tracker(cam.H, cam.W, (cam.fx, cam.fy, cam.cx, cam.cy), **VGA_PARAMS)
    t.set_stream(torch.cuda.current_stream())
    t.set_topology(pv.TOPO_QUADTREE)
    t.set_keyframe(torch.from_numpy(I0).to(dev), torch.from_numpy(N0).to(dev))
    for f in d_fr:
        t.track(f, 20, maps=False)
    t.close()
    run_adjoint(2, 10, 5, 1)
    # calibration: a plain device copy of a source evicted from the last-level
    # cache by a larger fill in between, so every source byte comes from HBM
    n = copy_mb * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    flush = torch.empty(2 * n, dtype=torch.float32, device=dev)
    for _ in range(3):
        flush.fill_(1.0)
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"probe done: copy calibration {copy_mb} MiB read + {copy_mb} MiB written per copy, 3 copies")


def run_central(args, g, n_frames: int = 2, irls_iters: int = 5):
    """The centralised IRLS Gauss-Newton baseline (Sec. 3.1, Sec. 4.4) on the
    same 640x480 frames: one global pose and per-pixel log-depths, the normal
    equations solved by FP64 preconditioned conjugate gradients (relative
    residual 1e-8). Reported per IRLS iteration."""
    import torch
    import paper_2606_03989_amd as pv
    cam, d_I0, d_N0, d_frames, d_normals, stream = g["inputs"]
    H, W = g["H"], g["W"]
    c = pv.Central(H, W, (cam.fx, cam.fy, cam.cx, cam.cy), max_cg=400, cg_tol=1e-8, **VGA_PARAMS)
    c.set_stream(stream)
    c.set_keyframe(d_I0, d_N0)
    c.track(d_frames[0], 1, maps=False)        # warm-up
    # the fused leg renders warmup + steps frames; a short run reuses them
    ms, cg = 0.0, 0
    for i in range(n_frames):
        r = c.track(d_frames[(1 + i) % len(d_frames)], irls_iters, maps=True, out_device=True)
        ms += c.last_ms()
        cg += r["cg_iters"]
    torch.cuda.synchronize()
    c.close()
    per_iter = ms / (n_frames * irls_iters)
    log(f"centralised IRLS: {per_iter:.2f} ms per IRLS iteration, {cg / (n_frames * irls_iters):.0f} CG iterations each")
    return dict(ms_per_irls_iteration=round(per_iter, 3), cg_iterations_per_irls=round(cg / (n_frames * irls_iters), 1),
                cg_tol=1e-8, frames=n_frames, irls_iterations_per_frame=irls_iters,
                Mpixel_iter_per_s=round(H * W / (per_iter / 1e3) / 1e6, 1),
                gbp_iteration_ms=round(g["pass_us"] / 1e3, 4))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--per-factor-steps", type=int, default=3)
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--probe", action="store_true", help="short run for hardware counters; no JSON line")
    ap.add_argument("--noise-sweep", action="store_true",
                    help="tracking accuracy under sensor noise (clean, Gaussian, mild, strong); its own JSON line")
    ap.add_argument("--batch-frames", type=int, default=49,
                    help="tracked frames per 50-frame sequence of the 64-sequence batch (at most 49: frame 0 is the "
                         "keyframe); 2 warm up, the rest are timed (0: skip)")
    ap.add_argument("--batch-seqs", type=int, default=64)
    ap.add_argument("--batch-kf-frames", type=int, default=16,
                    help="frames per keyframe in the batch leg (re-anchoring inside the timed steps)")
    ap.add_argument("--no-quadtree", dest="quadtree", action="store_false",
                    help="skip the quadtree-topology leg on the same frames")
    ap.add_argument("--transfer-check", action="store_true",
                    help="re-anchoring with and without keyframe depth transfer; its own JSON line")
    ap.add_argument("--compare-solvers", action="store_true",
                    help="centralised IRLS against distributed GBP on the slow-motion 256x256 scene; its own JSON line")
    ap.add_argument("--no-central", dest="central", action="store_false",
                    help="skip the centralised IRLS Gauss-Newton leg on the same frames")
    ap.add_argument("--adjoint-frames", type=int, default=29,
                    help="target frames of the forward+adjoint leg (the 30-frame sequence after its keyframe; 0: skip)")
    args = ap.parse_args()
    if args.probe:
        probe()
        return
    if args.noise_sweep:
        noise_sweep()
        return
    if args.compare_solvers:
        compare_solvers()
        return
    if args.transfer_check:
        transfer_check()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (single-GPU build)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("need --steps >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    g = run_gpu(args)
    quadtree = run_quadtree(args, g) if args.quadtree else None
    central = run_central(args, g) if args.central else None
    batched = (run_batch(args.batch_seqs, args.batch_frames, 15, 2, kf_frames=args.batch_kf_frames)
               if args.batch_frames > 2 else None)
    adjoint = run_adjoint(args.adjoint_frames, 30, 10, 2) if args.adjoint_frames > 0 else None
    cpu = None if args.no_cpu else cpu_baseline(args.cpu_iters)
    out = {
        "metric": "GBP Mpixel-iter/s at 640x480 + % HBM roofline; batched & fwd+adjoint vs plain",
        "value": round(g["value"], 1),
        "unit": "Mpixel-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(g["elapsed"] * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "storage_dtype": "f32",
        "precision": "fp32 storage, fp64 arithmetic",
        "data": "synthetic",
        "config": {"workload": "vga640x480 piecewise-planar sequence, 20 GBP iterations per frame, fused schedule",
                   "H": g["H"], "W": g["W"], "iters_per_frame": g["iters"], "state": "fp32 SoA, 123 planes",
                   "sigma_P": VGA_PARAMS["sigma_P"], "huber_k": VGA_PARAMS["huber_k"]},
        "roofline": g["roofline"],
        "cpu_baseline": cpu,
        "per_factor": g["per_factor"],
        "frame_step": g["frame_step"],
        "batched": batched,
        "forward_adjoint": adjoint,
        "quadtree": quadtree,
        "centralised": central,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
