"""GPU centralised IRLS Gauss-Newton baseline (Sec. 3.1, Sec. 4.4) against
the oracle's exact sparse solve (oracle/centralised.py), through the C-ABI."""

import math

import numpy as np
import pytest

import synth
from oracle.centralised import Centralised
from parity import sequence_workload

pytestmark = pytest.mark.gpu


def f32(x):
    return float(np.float32(x))


def _pair(w, max_cg=3000, cg_tol=1e-12, **kw):
    import paper_2606_03989_amd as pv
    cam = w["cam"]
    K = tuple(f32(k) for k in (cam.fx, cam.fy, cam.cx, cam.cy))
    kw = {k: f32(v) for k, v in kw.items()}
    c = pv.Central(cam.H, cam.W, K, max_cg=max_cg, cg_tol=cg_tol, **kw)
    c.set_keyframe(w["I_s"], w["N_s"])
    full = dict(sigma_D=f32(5e-3), sigma_P=f32(1.0), sigma_N=f32(1e-3), huber_k=f32(400.0))
    full.update({k: v for k, v in kw.items() if k in full})
    o = Centralised(cam.H, cam.W, K, w["I_s"], w["N_s"], **full)
    return c, o


def _tiny():
    p = synth.tiny_pair(0)
    return dict(cam=p["cam"], I_s=p["I_s"], N_s=p["normals_s"], frames=[p["I_t"]])


def _agree(name, xg, lg, xo, lo, x0, l0, rel=1e-6):
    dp = np.abs(xg - xo).max() / max(np.abs(xo - x0).max(), 1e-12)
    dl = np.abs(lg.reshape(-1) - lo).max() / max(np.abs(lo - l0.reshape(-1)).max(), 1e-12)
    print(f"{name}: pose diff / step {dp:.2e}, log-depth diff / step {dl:.2e}", flush=True)
    assert dp <= rel and dl <= rel


@pytest.mark.parametrize("huber_k", [400.0, 1.0])
def test_single_irls_step_from_a_set_point(huber_k):
    w = _tiny()
    cam = w["cam"]
    c, o = _pair(w, sigma_P=0.1, sigma_N=1e-2, sigma_D=2e-2, huber_k=huber_k, init_inv_depth=0.4)
    rng = np.random.default_rng(0)
    x0 = rng.normal(0, 0.005, 6)
    l0 = -math.log(0.4) + rng.normal(0, 0.05, (cam.H, cam.W))
    c.set_point(x0, l0)
    xg0, lg0 = c.get_point()
    assert np.array_equal(xg0, x0) and np.array_equal(lg0, l0)
    r = c.track(w["frames"][0], 1)
    o.set_frame(w["frames"][0])
    xo, lo = o.iterate(x0, l0.reshape(-1), 1)
    xg, lg = c.get_point()
    print(f"CG iterations {r['cg_iters']}, residual {r['last_rel_residual']:.1e}", flush=True)
    assert r["last_rel_residual"] <= 1e-12 and r["flags"] == 0
    _agree(f"tiny k={huber_k}", xg, lg, xo, lo, x0, l0)
    np.testing.assert_allclose(r["inv_depth"], np.exp(-lg), rtol=1e-6)


def test_irls_iterations_256():
    w = sequence_workload("ppa256", 1)
    cam = w["cam"]
    c, o = _pair(w, cg_tol=1e-11, sigma_P=0.01, huber_k=400.0)
    n = 5
    r = c.track(w["frames"][0], n)
    o.set_frame(w["frames"][0])
    x0, l0 = np.zeros(6), np.zeros((cam.H, cam.W))
    xo, lo = o.iterate(x0, l0.reshape(-1), n)
    xg, lg = c.get_point()
    print(f"256x256, {n} IRLS iterations: {r['cg_iters']} CG iterations, {c.last_ms():.1f} ms", flush=True)
    _agree("ppa256 5 iterations", xg, lg, xo, lo, x0, l0, rel=1e-5)


def test_vga_one_step():
    w = sequence_workload("vga", 1)
    cam = w["cam"]
    c, o = _pair(w, cg_tol=1e-11, **w["kw"])
    r = c.track(w["frames"][0], 1)
    o.set_frame(w["frames"][0])
    x0, l0 = np.zeros(6), np.zeros((cam.H, cam.W))
    xo, lo = o.iterate(x0, l0.reshape(-1), 1)
    xg, lg = c.get_point()
    print(f"640x480 one IRLS step: {r['cg_iters']} CG iterations, {c.last_ms():.1f} ms, valid {r['valid_fraction']:.4f}",
          flush=True)
    _agree("vga one step", xg, lg, xo, lo, x0, l0, rel=1e-5)


def test_errors():
    import paper_2606_03989_amd as pv
    w = _tiny()
    cam = w["cam"]
    K = (cam.fx, cam.fy, cam.cx, cam.cy)
    with pytest.raises(pv.PixvodError):
        pv.Central(cam.H, cam.W, K, max_cg=0)
    with pytest.raises(pv.PixvodError):
        pv.Central(1, cam.W, K)
    c = pv.Central(cam.H, cam.W, K)
    with pytest.raises(pv.PixvodError):
        c.track(w["frames"][0], 1)           # no keyframe
    c.set_keyframe(w["I_s"], w["N_s"])
    r = c.track(w["frames"][0], 0)           # no iteration: the point stays
    assert np.all(r["xi"] == 0) and r["cg_iters"] == 0
    c.close()
