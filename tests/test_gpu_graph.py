"""The captured frame step of one context (a HIP graph per starting buffer,
replayed) against launching every pass on its own: bit-identical states,
poses and maps across replays, re-captures after a changed kernel argument
(sigma map, iteration count) and a keyframe change, with and without
profiling event nodes in the graph."""

import time

import numpy as np
import pytest

from parity import make_tracker, sequence_workload

pytestmark = pytest.mark.gpu


def _run(w, graph, plan, profile=False):
    t = make_tracker(w)
    t.set_graph(graph)
    t.profile(profile)
    out = []
    a = time.perf_counter()
    for step in plan:
        if step[0] == "track":
            r = t.track(w["frames"][step[1]], step[2])
            out.append((r["xi"], r["inv_depth"], r["inv_depth_var"], r["flags"], t.get_state()))
        elif step[0] == "sigma":
            t.set_sigma_map(step[1])
        else:
            t.set_keyframe(w["frames"][step[1]], w["N_s"])
    dt = time.perf_counter() - a
    counts = [t.profile_read(k)[1] for k in range(3)] if profile else None
    t.close()
    return out, counts, dt


@pytest.mark.parametrize("profile", [False, True])
def test_graph_replay_equals_unrolled_passes(profile):
    w = sequence_workload("ppa256", 4)
    rng = np.random.default_rng(5)
    sig = rng.uniform(4e-3, 6e-3, (w["cam"].H, w["cam"].W)).astype(np.float32)
    # n = 5 keeps the starting buffer (replays of one graph), n = 4 flips it
    plan = [("track", 0, 5), ("track", 1, 5), ("sigma", sig), ("track", 2, 5), ("track", 3, 4),
            ("track", 0, 4), ("keyframe", 3), ("track", 1, 4), ("track", 2, 4), ("track", 3, 5)]
    ref, cref, tr = _run(w, False, plan, profile)
    got, cgot, tg = _run(w, True, plan, profile)
    n_tracks = sum(1 for s in plan if s[0] == "track")
    print(f"profile {profile}: {n_tracks} frames, graph {tg * 1e3:.1f} ms, unrolled {tr * 1e3:.1f} ms "
          f"(first captures included); launch counts iterate/final/prologue {cgot} vs {cref}", flush=True)
    assert len(got) == len(ref) == n_tracks
    for k, (a, b) in enumerate(zip(got, ref)):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y, err_msg=f"frame step {k}")
    if profile:
        iters = sum(s[2] for s in plan if s[0] == "track")
        assert cref == [iters - n_tracks, n_tracks, n_tracks]
        assert cgot == cref


