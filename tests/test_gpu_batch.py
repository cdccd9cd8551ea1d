"""Batched tracking (many sequences of mixed resolution per launch): every
sequence of a batch is checked against the FP64 oracle (one iteration from an
identical state, and a free-running frame), the batch must reproduce
per-sequence contexts bit for bit, for every tile shape, and its frame-step
graph must replay consistently."""

import numpy as np
import pytest

import synth
from parity import (check_free_running, check_iteration, from_oracle, iteration_spread, make_oracle,
                    oracle_spread, plane_errors, to_oracle)

pytestmark = pytest.mark.gpu

PARAMS = dict(sigma_P=0.01, huber_k=10.0, init_inv_depth=0.5)


def _seq_inputs(shapes, n_frames, seed=0):
    """Small textured sequences: a keyframe and frames with sub-pixel motion."""
    out = []
    for k, (H, W) in enumerate(shapes):
        rv = [0.001 * (k % 3), -0.002, 0.001]
        tr = [0.004 + 0.001 * k, -0.002, 0.003]
        frames = []
        for f in range(n_frames):
            s = (f + 1) / n_frames
            p = synth.tiny_pair(seed + k, H=H, W=W, inv_depth=0.5 + 0.1 * (k % 4),
                                rotvec=[x * s for x in rv], trans=[x * s for x in tr])
            frames.append(p["I_t"])
        out.append(dict(cam=p["cam"], I_s=p["I_s"], N_s=p["normals_s"], frames=frames))
    return out


def _K(cam):
    return (cam.fx, cam.fy, cam.cx, cam.cy)


def _make_batch(seqs, tile=None):
    import paper_2606_03989_amd as pv
    b = pv.Batch([(s["cam"].H, s["cam"].W) for s in seqs], [_K(s["cam"]) for s in seqs], **PARAMS)
    if tile:
        b.set_tile(*tile)
    b.set_keyframes(list(range(len(seqs))), [s["I_s"] for s in seqs], [s["N_s"] for s in seqs])
    return b


SHAPES = [(24, 32), (29, 37), (48, 64), (7, 130)]


def _oracle_workload(s, frame, iters):
    return dict(cam=s["cam"], I_s=s["I_s"], N_s=s["N_s"], frames=[frame], iters=iters, kw=dict(PARAMS))


def test_batch_against_oracle():
    # free-running first frame of every sequence (15 iterations, the batched
    # workload's count), then one iteration of every sequence from a state
    # loaded identically into batch and oracle (all 123 planes)
    seqs = _seq_inputs(SHAPES, 2)
    b = _make_batch(seqs)
    iters = 15
    rb = b.track([s["frames"][0] for s in seqs], iters, maps=True)
    for i, s in enumerate(seqs):
        w = _oracle_workload(s, s["frames"][0], iters)
        o = make_oracle(w)
        ro = o.track(s["frames"][0], iters)
        spread = oracle_spread(w, s["frames"][0], iters, ref=ro)
        check_free_running(rb[i], ro, spread, f"batch sequence {i} ({s['cam'].H}x{s['cam'].W}) frame 1")
        assert rb[i]["frames_since_keyframe"] == ro["frames_since_keyframe"] == 1
        o.close()
    starts = []
    for i, s in enumerate(seqs):
        w = _oracle_workload(s, s["frames"][1], iters)
        o = make_oracle(w)
        o.track(s["frames"][1], 3)
        s32 = from_oracle(o.get_state())
        b.set_state(i, s32)
        np.testing.assert_array_equal(b.get_state(i), s32)
        starts.append((w, s32))
        o.close()
    b.track([s["frames"][1] for s in seqs], 1)
    for i, (w, s32) in enumerate(starts):
        o = make_oracle(w)
        o.set_state(to_oracle(s32))
        o.set_frame(w["frames"][0])
        o.iterate(1)
        err = plane_errors(b.get_state(i), from_oracle(o.get_state()))
        spread = iteration_spread(w, s32, w["frames"][0]) if err.max() > 1e-5 else None
        check_iteration(err, spread, f"batch sequence {i} one iteration")
        o.close()


def test_batch_equals_per_sequence_contexts():
    import paper_2606_03989_amd as pv
    seqs = _seq_inputs(SHAPES, 3)
    b = _make_batch(seqs)
    singles = []
    for s in seqs:
        t = pv.Tracker(s["cam"].H, s["cam"].W, _K(s["cam"]), **PARAMS)
        t.set_keyframe(s["I_s"], s["N_s"])
        singles.append(t)
    for f in range(3):
        rb = b.track([s["frames"][f] for s in seqs], 6, maps=True)
        for i, (s, t) in enumerate(zip(seqs, singles)):
            rs = t.track(s["frames"][f], 6)
            np.testing.assert_array_equal(b.get_state(i), t.get_state())
            # both reduce the pose planes over the same 64 x 4 tiles in the
            # same order, so the pose means agree bit for bit
            np.testing.assert_array_equal(rb[i]["xi"], rs["xi"])
            np.testing.assert_array_equal(rb[i]["inv_depth"], rs["inv_depth"])
            assert rb[i]["frames_since_keyframe"] == rs["frames_since_keyframe"] == f + 1
            assert rb[i]["flags"] == rs["flags"]
    print("batch == per-sequence contexts over 3 graph-replayed frame steps", flush=True)


@pytest.mark.parametrize("tile", [(64, 4), (16, 16), (32, 1), (128, 2)])
def test_tile_shape_does_not_change_results(tile):
    seqs = _seq_inputs(SHAPES, 2)
    ref = _make_batch(seqs, (64, 1))
    b = _make_batch(seqs, tile)
    for f in range(2):
        rr = ref.track([s["frames"][f] for s in seqs], 4, maps=True)
        rb = b.track([s["frames"][f] for s in seqs], 4, maps=True)
        # the pose statistics use fixed 64 x 4 tiles whatever the work-item
        # shape, so the outputs agree bit for bit as well
        for i in range(len(seqs)):
            np.testing.assert_array_equal(rb[i]["xi"], rr[i]["xi"])
            np.testing.assert_array_equal(rb[i]["T_world"], rr[i]["T_world"])
            np.testing.assert_array_equal(rb[i]["inv_depth"], rr[i]["inv_depth"])
    for i in range(len(seqs)):
        np.testing.assert_array_equal(b.get_state(i), ref.get_state(i))


def test_autotune_has_no_side_effects():
    seqs = _seq_inputs(SHAPES, 2)
    a = _make_batch(seqs)
    b = _make_batch(seqs)
    a.track([s["frames"][0] for s in seqs], 4)
    b.track([s["frames"][0] for s in seqs], 4)
    tx, ty = b.autotune(3)
    assert tx * ty <= 256
    print(f"autotuned tile {tx}x{ty}", flush=True)
    for i in range(len(seqs)):
        np.testing.assert_array_equal(a.get_state(i), b.get_state(i))
    a.track([s["frames"][1] for s in seqs], 4)
    b.track([s["frames"][1] for s in seqs], 4)
    for i in range(len(seqs)):
        np.testing.assert_array_equal(a.get_state(i), b.get_state(i))


def test_batch_errors():
    import paper_2606_03989_amd as pv
    seqs = _seq_inputs(SHAPES[:2], 1)
    b = pv.Batch([(s["cam"].H, s["cam"].W) for s in seqs], [_K(s["cam"]) for s in seqs], **PARAMS)
    with pytest.raises(pv.PixvodError) as e:
        b.track([s["frames"][0] for s in seqs], 3)
    assert e.value.code == pv.ESTATE
    with pytest.raises(pv.PixvodError) as e:
        b.set_tile(32, 16)
    assert e.value.code == pv.EINVAL
    with pytest.raises(pv.PixvodError) as e:
        pv.Batch([(2, 1)], [(10.0, 10.0, 1.0, 1.0)])
    assert e.value.code == pv.EINVAL


def test_full_size_mixed_batch_sampled_against_per_sequence():
    # the 64-sequence mixed-resolution batch (128x96, 256x256, 320x240, 640x480)
    # in the benchmark's launch configuration; sampled sequences are re-run
    # alone and must match bit for bit
    import paper_2606_03989_amd as pv
    from synth.scenes import batch_resolution
    rng = np.random.default_rng(5)
    shapes = [batch_resolution(s) for s in range(64)]
    Ks = [synth.Camera.default(H, W) for H, W in shapes]
    imgs, frames, normals = [], [], []
    for s, (H, W) in enumerate(shapes):
        yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
        base = synth.value_noise_texture(xx / 4.0, yy / 4.0, 100 + s, 3, 0.5)
        moved = synth.value_noise_texture((xx + 0.3) / 4.0, (yy - 0.2) / 4.0, 100 + s, 3, 0.5)
        imgs.append(base.astype(np.float32))
        frames.append(moved.astype(np.float32))
        n = np.zeros((H, W, 3), np.float32)
        n[..., 2] = -1.0
        normals.append(n)
    b = pv.Batch(shapes, [_K(k) for k in Ks], **PARAMS)
    b.set_keyframes(list(range(64)), imgs, normals)
    rb = b.track(frames, 3)
    for s in (0, 1, 2, 3, 37, 63):
        H, W = shapes[s]
        t = pv.Tracker(H, W, _K(Ks[s]), **PARAMS)
        t.set_keyframe(imgs[s], normals[s])
        rs = t.track(frames[s], 3)
        np.testing.assert_array_equal(rb[s]["xi"], rs["xi"])
        np.testing.assert_array_equal(b.get_state(s), t.get_state())
        t.close()
    print(f"64-sequence batch frame step {b.last_step_ms():.2f} ms", flush=True)
    b.close()


def test_device_reanchoring_equals_host_reanchoring():
    # keyframe test and re-anchoring inside the captured frame step (device
    # flag, predicated kernel) against per-sequence contexts re-anchored from
    # the host when their flag fires; every second frame is due
    import paper_2606_03989_amd as pv
    seqs = _seq_inputs(SHAPES, 5)
    params = dict(PARAMS, kf_max_frames=2)
    b = pv.Batch([(s["cam"].H, s["cam"].W) for s in seqs], [_K(s["cam"]) for s in seqs], **params)
    b.set_keyframes(list(range(len(seqs))), [s["I_s"] for s in seqs], [s["N_s"] for s in seqs])
    singles = []
    for s in seqs:
        t = pv.Tracker(s["cam"].H, s["cam"].W, _K(s["cam"]), **params)
        t.set_keyframe(s["I_s"], s["N_s"])
        singles.append(t)
    n_due = 0
    for f in range(5):
        rb = b.track([s["frames"][f] for s in seqs], 4, maps=True, normals=[s["N_s"] for s in seqs])
        for i, (s, t) in enumerate(zip(seqs, singles)):
            rs = t.track(s["frames"][f], 4)
            assert rb[i]["flags"] == rs["flags"] and rb[i]["frames_since_keyframe"] == rs["frames_since_keyframe"]
            np.testing.assert_array_equal(rb[i]["inv_depth"], rs["inv_depth"])
            np.testing.assert_array_equal(rb[i]["T_world"], rs["T_world"])
            if rs["flags"] & pv.KEYFRAME_DUE:
                n_due += 1
                t.set_keyframe(s["frames"][f], s["N_s"])
            np.testing.assert_array_equal(b.get_state(i), t.get_state())
    assert n_due >= 2 * len(seqs)
    print(f"device re-anchoring: {n_due} re-anchorings over 5 frames, batch == host-side re-anchoring", flush=True)


@pytest.mark.parametrize("reanchor", [False, True])
def test_persistent_iteration_block_equals_launch_per_pass(reanchor):
    import paper_2606_03989_amd as pv
    seqs = _seq_inputs(SHAPES, 3)
    params = dict(PARAMS, kf_max_frames=2)
    batches = []
    for persistent in (False, True):
        b = pv.Batch([(s["cam"].H, s["cam"].W) for s in seqs], [_K(s["cam"]) for s in seqs], **params)
        b.set_persistent(persistent)
        b.set_keyframes(list(range(len(seqs))), [s["I_s"] for s in seqs], [s["N_s"] for s in seqs])
        batches.append(b)
    for f in range(3):
        kw = dict(normals=[s["N_s"] for s in seqs]) if reanchor else {}
        ra = batches[0].track([s["frames"][f] for s in seqs], 5, **kw)
        rp = batches[1].track([s["frames"][f] for s in seqs], 5, **kw)
        for i in range(len(seqs)):
            np.testing.assert_array_equal(ra[i]["xi"], rp[i]["xi"])
            assert ra[i]["flags"] == rp[i]["flags"]
            np.testing.assert_array_equal(batches[0].get_state(i), batches[1].get_state(i))
    print(f"persistent iteration block == one launch per pass (re-anchoring {reanchor}); "
          f"step {batches[1].last_step_ms():.3f} ms against {batches[0].last_step_ms():.3f} ms", flush=True)
