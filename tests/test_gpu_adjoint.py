"""Hand-written adjoint of the unrolled iterations against the FP64 oracle.

The reference gradient is the oracle's: central differences (relative step
1e-6) of unrolled FP64 tracking. The unrolled iteration is chaotic beyond a
few dozen iterations from a cold keyframe state on these sequences (a one-ulp
change of the input frames moves the oracle's own difference quotients by
O(1) after 30 iterations), so the comparisons use horizons where that
sensitivity is small: two frames of ten iterations on the 24x24 crop, one
frame of ten iterations at 320x240. Tolerances follow the measured spread of
the oracle's gradient under one-ulp input perturbations (1e-5 for sigma_N,
4e-3 for the Huber threshold on the crop; 5e-3 at full size).
"""

import numpy as np
import pytest
import torch

from parity import diff_crop_workload, diff_full_workload, from_oracle, make_unroll, make_unrolled_oracle, to_oracle

pytestmark = pytest.mark.gpu


def _gpu_grads(w, n_iters, ckpt, frames=None):
    u = make_unroll(w, n_iters, ckpt)
    fr = np.stack(frames if frames is not None else w["frames"]).astype(np.float32)
    xi, rho = u.forward(fr, w["sigma_map"], w["sigma_N"], w["huber_k"])
    g, gN, gk = u.backward(w["cxi"], w["crho"])
    u.close()
    return xi, rho, g, gN, gk


def test_crop_gradients_match_oracle_differences():
    w = diff_crop_workload(24, 2)
    xi, rho, g, gN, gk = _gpu_grads(w, 10, 4)
    o = make_unrolled_oracle(w, 10)
    out = o.outputs()
    assert np.abs(xi - out["xi"]).max() <= 1e-5
    fN, fk = o.d_sigma_N(w["cxi"], w["crho"]), o.d_huber_k(w["cxi"], w["crho"])
    print(f"sigma_N: adjoint {gN:.9e} oracle {fN:.9e}; huber_k: adjoint {gk:.9e} oracle {fk:.9e}", flush=True)
    assert abs(gN - fN) <= 1e-3 * abs(fN)
    assert abs(gk - fk) <= 2e-2 * abs(fk)
    # sigma map: an 8x8 block at the image corner, 40 random entries
    rng = np.random.default_rng(0)
    entries = [(v, u) for v in range(8) for u in range(8)]
    entries += [tuple(x) for x in rng.integers(0, 24, size=(40, 2))]
    fd = np.array([o.d_sigma_entry(w["cxi"], w["crho"], v, u) for v, u in entries])
    ad = np.array([g[v, u] for v, u in entries], np.float64)
    err = np.abs(ad - fd)
    scale = np.abs(fd).max()
    print(f"sigma map: {len(entries)} entries, max |adj - fd| {err.max():.3e} of max |fd| {scale:.3e}", flush=True)
    assert np.all(err <= 1e-3 * scale + 1e-3 * np.abs(fd))
    # every entry at once along a random direction
    d = rng.uniform(-1.0, 1.0, (24, 24))
    fdd = o.d_direction(w["cxi"], w["crho"], d, 0.0, 0.0)
    add = float(np.sum(g.astype(np.float64) * d * w["sigma_map"].astype(np.float64)))
    print(f"directional: adjoint {add:.9e} oracle {fdd:.9e}", flush=True)
    assert abs(add - fdd) <= 1e-3 * abs(fdd)


def test_full_size_directional_derivative():
    # 320x240, one frame of ten iterations, checkpoints every 4
    w = diff_full_workload(1)
    xi, rho, g, gN, gk = _gpu_grads(w, 10, 4)
    o = make_unrolled_oracle(w, 10)
    rng = np.random.default_rng(1)
    d = rng.uniform(-1.0, 1.0, w["sigma_map"].shape)
    dN, dk = 0.7, -0.4
    fdd = o.d_direction(w["cxi"], w["crho"], d, dN, dk)
    add = (float(np.sum(g.astype(np.float64) * d * w["sigma_map"].astype(np.float64))) + gN * dN * w["sigma_N"] +
           gk * dk * w["huber_k"])
    print(f"320x240 directional derivative: adjoint {add:.9e} oracle {fdd:.9e}", flush=True)
    assert abs(add - fdd) <= 5e-3 * abs(fdd)


def test_teacher_forced_one_iteration_full_size():
    # 320x240: both sides start from the oracle's state after ten iterations
    # of frame 1 (rounded to the FP32 state) and run one iteration of frame 2;
    # a single iteration is smooth in the parameters, so the reverse kernels
    # meet the oracle's FP64 differences closely at full size
    import oracle
    from oracle.gradient import UnrolledOracle
    w = diff_full_workload(2)
    cam = w["cam"]
    o = oracle.Oracle(oracle.config_for_camera(cam, sigma_N=w["sigma_N"], huber_k=w["huber_k"], **w["kw"]))
    o.set_sigma_D_map(w["sigma_map"])
    o.set_keyframe(w["I_s"], w["N_s"])
    o.track(w["frames"][0], 10)
    start32 = from_oracle(o.get_state())
    o.close()
    frame = w["frames"][1]
    cxi, crho = w["cxi"][1:2], w["crho"][1:2]
    u = make_unroll(dict(w, frames=[frame]), 1, 1)
    u.set_state(start32)
    xi, rho = u.forward(np.stack([frame]).astype(np.float32), w["sigma_map"], w["sigma_N"], w["huber_k"])
    g, gN, gk = u.backward(cxi, crho)
    u.close()
    orc = UnrolledOracle(cam, w["I_s"], w["N_s"], [frame], 1, w["sigma_map"], w["sigma_N"], w["huber_k"],
                         start=to_oracle(start32), **w["kw"])
    out = orc.outputs()
    dxi = np.abs(xi - out["xi"]).max()
    print(f"one iteration from the oracle's state: pose {dxi:.2e}", flush=True)
    assert dxi <= 1e-5
    fN, fk = orc.d_sigma_N(cxi, crho), orc.d_huber_k(cxi, crho)
    eN, ek = abs(gN - fN) / abs(fN), abs(gk - fk) / abs(fk)
    print(f"sigma_N: adjoint {gN:.9e} differences {fN:.9e} (rel {eN:.1e}); "
          f"huber_k: adjoint {gk:.9e} differences {fk:.9e} (rel {ek:.1e})", flush=True)
    rng = np.random.default_rng(2)
    entries = [tuple(x) for x in rng.integers(0, (cam.H, cam.W), size=(24, 2))]
    fd = np.array([orc.d_sigma_entry(cxi, crho, v, u_) for v, u_ in entries])
    ad = np.array([g[v, u_] for v, u_ in entries], np.float64)
    scale = np.abs(fd).max()
    err = np.abs(ad - fd)
    print(f"sigma map: {len(entries)} entries, max |adj - fd| {err.max():.3e} of max |fd| {scale:.3e}", flush=True)
    d = rng.uniform(-1.0, 1.0, (cam.H, cam.W))
    dN, dk = 0.7, -0.4
    fdd = orc.d_direction(cxi, crho, d, dN, dk)
    add = (float(np.sum(g.astype(np.float64) * d * w["sigma_map"].astype(np.float64))) + gN * dN * w["sigma_N"] +
           gk * dk * w["huber_k"])
    edd = abs(add - fdd) / abs(fdd)
    print(f"directional: adjoint {add:.9e} differences {fdd:.9e} (rel {edd:.1e})", flush=True)
    assert eN <= 1e-4 and ek <= 1e-3
    assert np.all(err <= 1e-4 * scale + 1e-4 * np.abs(fd))
    assert edd <= 1e-4


def test_checkpoint_interval_does_not_change_gradients():
    w = diff_crop_workload(40, 2)
    ref = _gpu_grads(w, 10, 1)
    for ck in (3, 10):
        got = _gpu_grads(w, 10, ck)
        np.testing.assert_array_equal(got[0], ref[0])
        np.testing.assert_array_equal(got[2], ref[2])
        assert got[3] == ref[3] and got[4] == ref[4]


def test_forward_equals_tracker():
    import paper_2606_03989_amd as pv
    from parity import K_of
    w = diff_crop_workload(48, 2)
    xi, rho, *_ = _gpu_grads(w, 10, 4)
    cam = w["cam"]
    t = pv.Tracker(cam.H, cam.W, K_of(cam), sigma_N=w["sigma_N"], huber_k=w["huber_k"], **w["kw"])
    t.set_sigma_map(w["sigma_map"])
    t.set_keyframe(w["I_s"], w["N_s"])
    for f, fr in enumerate(w["frames"]):
        r = t.track(fr, 10)
        np.testing.assert_allclose(xi[f], r["xi"], rtol=1e-12, atol=1e-15)
        np.testing.assert_array_equal(rho[f], r["inv_depth"])
    t.close()


def test_backward_is_repeatable_and_linear():
    w = diff_crop_workload(32, 2)
    u = make_unroll(w, 10, 4)
    fr = np.stack(w["frames"]).astype(np.float32)
    u.forward(fr, w["sigma_map"], w["sigma_N"], w["huber_k"])
    a = u.backward(w["cxi"], w["crho"])
    b = u.backward(w["cxi"], w["crho"])
    np.testing.assert_array_equal(a[0], b[0])
    assert a[1] == b[1] and a[2] == b[2]
    z = u.backward(None, None)
    assert np.all(z[0] == 0) and z[1] == 0 and z[2] == 0
    # the adjoint is linear in the output cotangents
    x1 = u.backward(w["cxi"], None)
    x2 = u.backward(None, w["crho"])
    np.testing.assert_allclose(x1[0] + x2[0], a[0], rtol=1e-4, atol=1e-6 * np.abs(a[0]).max())
    assert abs(x1[1] + x2[1] - a[1]) <= 1e-5 * abs(a[1]) + 1e-12
    u.close()


def test_errors():
    import paper_2606_03989_amd as pv
    w = diff_crop_workload(24, 1)
    cam = w["cam"]
    with pytest.raises(pv.PixvodError) as e:
        pv.Unrolled(cam.H, cam.W, (30.0, 30.0, 12.0, 12.0), n_iters=0, max_frames=1)
    assert e.value.code == pv.EINVAL
    with pytest.raises(pv.PixvodError) as e:
        pv.Unrolled(cam.H, cam.W, (30.0, 30.0, 12.0, 12.0), n_iters=5, max_frames=1, damping=0.5)
    assert e.value.code == pv.EINVAL
    u = pv.Unrolled(cam.H, cam.W, (30.0, 30.0, 12.0, 12.0), n_iters=5, max_frames=1)
    with pytest.raises(pv.PixvodError) as e:
        u.backward(None, None)
    assert e.value.code == pv.ESTATE
    fr = np.stack(w["frames"]).astype(np.float32)
    with pytest.raises(pv.PixvodError) as e:
        u.forward(fr, w["sigma_map"], 1e-3, 10.0)
    assert e.value.code == pv.ESTATE
    u.set_keyframe(w["I_s"], w["N_s"])
    with pytest.raises(pv.PixvodError) as e:
        u.forward(fr, w["sigma_map"], -1.0, 10.0)
    assert e.value.code == pv.EINVAL
    with pytest.raises(pv.PixvodError) as e:
        u.forward(np.concatenate([fr, fr]), w["sigma_map"], 1e-3, 10.0)
    assert e.value.code == pv.EINVAL
    u.close()


def test_autograd_function():
    import paper_2606_03989_amd as pv
    w = diff_crop_workload(32, 2)
    u = make_unroll(w, 10, 4)
    dev = torch.device("cuda")
    frames = torch.from_numpy(np.stack(w["frames"]).astype(np.float32)).to(dev)
    sig = torch.tensor(w["sigma_map"], device=dev, requires_grad=True)
    sN = torch.tensor(w["sigma_N"], dtype=torch.float64, device=dev, requires_grad=True)
    hk = torch.tensor(w["huber_k"], dtype=torch.float64, device=dev, requires_grad=True)
    xi, rho = pv.unrolled_track(u, frames, sig, sN, hk)
    # pose error numerator of the paper's relative error (translation part
    # on the tangent for brevity) plus the inverse-depth error
    xi_gt = torch.zeros_like(xi)
    rho_gt = torch.full_like(rho, 0.5)
    loss = ((xi - xi_gt) ** 2).sum() + ((rho - rho_gt) ** 2).mean()
    loss.backward()
    cx = (2 * (xi - xi_gt)).detach().cpu().numpy()
    cr = (2 * (rho - rho_gt) / rho.numel()).detach()
    g, gN, gk = u.backward(cx, cr)
    np.testing.assert_allclose(sig.grad.cpu().numpy(), g, rtol=1e-6, atol=1e-9 * np.abs(g).max())
    assert abs(sN.grad.item() - gN) <= 1e-9 * abs(gN) + 1e-15
    assert abs(hk.grad.item() - gk) <= 1e-9 * abs(gk) + 1e-15
    u.close()


def test_device_inputs_follow_torch_stream():
    # A float64 sigma map computed on the device by torch ops just before the
    # call, behind long-running work on torch's stream: the library's work is
    # ordered after it (it runs on torch's current stream), so the outputs equal
    # those of host inputs bit for bit, and the gradients those of the direct
    # backward call.
    import paper_2606_03989_amd as pv
    w = diff_crop_workload(32, 2)
    frames_np = np.stack(w["frames"]).astype(np.float32)
    u_host = make_unroll(w, 10, 4)
    xi_h, rho_h = u_host.forward(frames_np, w["sigma_map"], w["sigma_N"], w["huber_k"])
    u = make_unroll(w, 10, 4)
    dev = torch.device("cuda")
    frames = torch.from_numpy(frames_np).to(dev)
    x = torch.randn(3072, 3072, device=dev)
    for _ in range(6):
        x = torch.tanh(x @ x)                   # keeps torch's stream busy
    sig = torch.from_numpy(w["sigma_map"].astype(np.float64)).to(dev) + 0.0 * x[0, 0].double()
    sig.requires_grad_(True)
    sN = torch.tensor(w["sigma_N"], dtype=torch.float64, device=dev, requires_grad=True)
    hk = torch.tensor(w["huber_k"], dtype=torch.float64, device=dev, requires_grad=True)
    xi, rho = pv.unrolled_track(u, frames, sig, sN, hk)
    np.testing.assert_array_equal(xi.detach().cpu().numpy(), xi_h)
    np.testing.assert_array_equal(rho.detach().cpu().numpy(), rho_h)
    loss = (xi ** 2).sum() + ((rho - 0.5) ** 2).mean()
    loss.backward()
    cx = (2 * xi).detach().cpu().numpy()
    cr = (2 * (rho - 0.5) / rho.numel()).detach().cpu().numpy()
    g, gN, gk = u_host.backward(cx, cr)
    np.testing.assert_allclose(sig.grad.cpu().numpy(), g, rtol=1e-6, atol=1e-9 * np.abs(g).max())
    assert abs(sN.grad.item() - gN) <= 1e-9 * abs(gN) + 1e-15
    u.close()
    u_host.close()
