"""The allocation-free re-anchoring entry point
(pixvod_set_keyframe_transfer_noalloc, whose z-buffer is a static per-device
array) against the allocating one (pixvod_set_keyframe_transfer), through the
C-ABI: two calls in a row, the second on a smaller frame, must leave states
identical bit for bit."""

import numpy as np
import pytest

from parity import make_oracle, make_tracker, sequence_workload, tiny_workload

pytestmark = pytest.mark.gpu


def _moved_state(w, xi, seed):
    o = make_oracle(w)
    st = o.get_state()
    rng = np.random.default_rng(seed)
    st[..., :6] = xi + rng.normal(0, 1e-4, st[..., :6].shape)
    st[..., 6] = rng.uniform(-0.3, 1.0, st[..., 6].shape)
    o.close()
    return np.ascontiguousarray(np.transpose(st, (2, 0, 1)).astype(np.float32))


@pytest.mark.parametrize("where", ["host", "device"])
def test_noalloc_transfer_equals_allocating_entry_point(where):
    import torch
    xi = np.array([0.01, -0.02, 0.015, 0.08, -0.05, 0.1])
    # the larger frame first, then the smaller one: the static array keeps the
    # first call's contents, which the second must not see
    for k, w in enumerate((sequence_workload("ppa256", 1), tiny_workload())):
        s32 = _moved_state(w, xi, 10 + k)
        trackers = (make_tracker(w), make_tracker(w))
        for t in trackers:
            t.set_state(s32)
            t.track(w["frames"][0], 0)
        img, nrm = w["frames"][0], np.ascontiguousarray(w["N_s"])
        if where == "device":
            img, nrm = torch.from_numpy(img).cuda(), torch.from_numpy(nrm).cuda()
        trackers[0].set_keyframe(img, nrm, transfer_depth=True)
        trackers[1].set_keyframe(img, nrm, transfer_depth=True, noalloc=True)
        a, b = trackers[0].get_state(), trackers[1].get_state()
        moved = float(np.mean(a[6] != s32[6]))
        print(f"{w['cam'].H}x{w['cam'].W} ({where}): {moved:.3f} of the log-depths transferred; "
              f"states identical: {np.array_equal(a, b)}", flush=True)
        assert 0.3 < moved < 1.0
        np.testing.assert_array_equal(a, b)
        for t in trackers:
            t.close()


def test_noalloc_transfer_errors():
    import paper_2606_03989_amd as pv
    w = tiny_workload()
    t = make_tracker(w)
    with pytest.raises(pv.PixvodError) as e:              # no tracked frame yet
        t.set_keyframe(w["frames"][0], w["N_s"], transfer_depth=True, noalloc=True)
    assert e.value.code == pv.ESTATE
    t.close()
    # 1100 x 1920: H times the pitch exceeds the static array's 2^21 entries
    big = pv.Tracker(1100, 1920, (1800.0, 1800.0, 960.0, 550.0))
    img = np.zeros((1100, 1920), np.float32)
    nrm = np.zeros((1100, 1920, 3), np.float32)
    nrm[..., 2] = -1.0
    big.set_keyframe(img, nrm)
    big.track(img, 0)
    with pytest.raises(pv.PixvodError) as e:
        big.set_keyframe(img, nrm, transfer_depth=True, noalloc=True)
    assert e.value.code == pv.EINVAL
    big.set_keyframe(img, nrm, transfer_depth=True)       # the allocating entry point has no limit
    big.close()
