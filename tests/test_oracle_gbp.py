"""Pins of the oracle's GBP iteration against results fixed by the mathematics:
exact Gaussian inference (dense solves), the Gauss-Newton / IRLS fixed point,
an exact zero-residual scene, special cases and symmetries."""

import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def K_of(cam):
    return (cam.fx, cam.fy, cam.cx, cam.cy)


def make(p, **kw):
    cam = p["cam"]
    o = oracle.Oracle(oracle.config_for_camera(cam, **kw))
    o.set_keyframe(p["I_s"], p["normals_s"])
    o.set_frame(p["I_t"])
    return o


def test_default_strengths_are_the_papers():
    with open(os.path.join(GOLDEN, "paper_hyperparameters.json")) as f:
        g = json.load(f)
    cfg = oracle.default_config()
    for k in ("sigma_D", "sigma_P", "sigma_R", "sigma_N", "huber_k"):
        assert getattr(cfg, k) == g["values"][k]


# --- linear model: loopy GBP means are exact -------------------------------------

@pytest.mark.parametrize("seed", [3, 4])
def test_frozen_gbp_means_equal_dense_solve(seed):
    p = synth.tiny_pair(seed, H=5, W=6, lattice_px=2.0)
    cam = p["cam"]
    kw = dict(sigma_P=1e-2, sigma_R=1e-2, sigma_N=1e-2)
    o = make(p, init_inv_depth=0.4, frozen=1, **kw)
    st = o.get_state()
    rng = np.random.default_rng(seed)
    st[..., :6] = rng.normal(0, 0.003, size=st[..., :6].shape)
    st[..., 6] += rng.normal(0, 0.05, size=st[..., 6].shape)
    o.set_state(st)
    prob = dense.Problem(cam.H, cam.W, K_of(cam), p["I_s"], p["I_t"], p["normals_s"], **kw)
    ref = prob.solve_linear(st[..., :6].reshape(-1, 6), st[..., 6].reshape(-1))
    o.iterate(300)
    m = o.means().reshape(-1, 7)
    np.testing.assert_allclose(m, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_chain_marginal_covariances_are_exact():
    # a single image row is a chain (a tree): GBP marginals are exact
    p = synth.tiny_pair(3, H=24, W=32, lattice_px=2.0)
    cam = synth.Camera(1, 10, 9.4, 9.4, 4.5, 0.0)
    I_s = p["I_s"][12:13, 10:20].copy()
    I_t = p["I_t"][12:13, 10:20].copy()
    N = p["normals_s"][12:13, 10:20].copy()
    kw = dict(sigma_P=1e-2, sigma_R=1e-2, sigma_N=1e-2)
    o = oracle.Oracle(oracle.config_for_camera(cam, init_inv_depth=0.4, frozen=1, **kw))
    o.set_keyframe(I_s, N)
    o.set_frame(I_t)
    o.iterate(30)
    lam, eta = o.beliefs()
    st = o.get_state()
    prob = dense.Problem(1, 10, K_of(cam), I_s, I_t, N, **kw)
    L, h, nv = prob.assemble(st[..., :6].reshape(-1, 6), st[..., 6].reshape(-1))
    assert nv == 10
    S = np.linalg.inv(L)
    mu = S @ h
    for i in range(10):
        Si = S[7 * i:7 * i + 7, 7 * i:7 * i + 7]
        np.testing.assert_allclose(np.linalg.inv(lam[0, i]), Si, atol=1e-12 * np.abs(Si).max())
        np.testing.assert_allclose(np.linalg.solve(lam[0, i], eta[0, i]), mu[7 * i:7 * i + 7],
                                   atol=1e-12 * np.abs(mu).max())


# --- nonlinear model: relinearised GBP converges to the Gauss-Newton fixed point -----

@pytest.mark.parametrize("huber_k", [400.0, 1.0])
def test_relinearised_fixed_point_equals_dense_gauss_newton(huber_k):
    # the target camera moves backwards so every warp stays inside the image
    p = synth.tiny_pair(3, H=5, W=6, lattice_px=2.0, rotvec=[0, 0, 0], trans=[0.0, 0.0, -0.05])
    cam = p["cam"]
    kw = dict(sigma_P=1e-1, sigma_R=1e-2, sigma_N=1e-2, sigma_D=2e-2, huber_k=huber_k)
    o = make(p, init_inv_depth=0.4, **kw)
    prob = dense.Problem(cam.H, cam.W, K_of(cam), p["I_s"], p["I_t"], p["normals_s"], **kw)
    st0 = o.get_state()
    tau, ell = prob.gauss_newton(st0[..., :6].reshape(-1, 6), st0[..., 6].reshape(-1), 15)
    L, h, nv = prob.assemble(tau, ell)
    assert nv == cam.H * cam.W and np.abs(h).max() < 1e-3      # GN has converged
    o.iterate(1500)
    assert np.abs(o.means()).max() < 1e-7                      # so has GBP
    st = o.get_state()
    np.testing.assert_allclose(st[..., :6].reshape(-1, 6), tau, atol=5e-8)
    np.testing.assert_allclose(st[..., 6].reshape(-1), ell, atol=5e-8)


# --- exact zero-residual scene ----------------------------------------------------

def _zero_residual(p):
    cam = p["cam"]
    tau_true = oracle.se3_log(p["T_ts"])
    ell_true = np.full((cam.H, cam.W), math.log(2.0))      # plane at inverse depth 0.5
    I_s0 = dense.zero_residual_source(p["I_t"], K_of(cam), tau_true, ell_true, p["I_s"])
    return tau_true, I_s0


def test_truth_is_an_exact_fixed_point(tiny):
    cam = tiny["cam"]
    tau_true, I_s0 = _zero_residual(tiny)
    cfg = oracle.config_for_camera(cam, prior_xi=tau_true, prior_log_depth=math.log(2.0), init_inv_depth=0.5)
    o = oracle.Oracle(cfg)
    o.set_keyframe64(I_s0, tiny["normals_s"])
    o.set_frame64(tiny["I_t"].astype(np.float64))
    st = o.get_state()
    st[..., :6] = tau_true
    o.set_state(st)
    assert o.energy() < 1e-18
    o.iterate(20)
    st = o.get_state()
    assert np.abs(st[..., :6] - tau_true).max() < 1e-12
    assert np.abs(st[..., 6] - math.log(2.0)).max() < 1e-12
    assert np.abs(o.means()).max() < 1e-12


def test_zero_residual_scene_converges_to_truth(tiny):
    cam = tiny["cam"]
    tau_true, I_s0 = _zero_residual(tiny)
    cfg = oracle.config_for_camera(cam, prior_xi=tau_true, prior_log_depth=math.log(2.0),
                                   init_inv_depth=0.3, sigma_P=0.01)
    o = oracle.Oracle(cfg)
    o.set_keyframe64(I_s0, tiny["normals_s"])
    o.set_frame64(tiny["I_t"].astype(np.float64))
    energies, derr = [o.energy()], []
    for _ in range(6):
        o.iterate(50)
        st = o.get_state()
        energies.append(o.energy())
        derr.append(np.abs(np.exp(-st[..., 6]) - 0.5).max())
    assert all(b < a for a, b in zip(energies, energies[1:]))
    assert all(b < a for a, b in zip(derr, derr[1:]))
    assert derr[-1] < 2e-5 and energies[-1] < 1e-4 * energies[0]
    xi = st[..., :6].reshape(-1, 6).mean(0)
    assert np.abs(xi - tau_true).max() < 2e-3


# --- special cases -----------------------------------------------------------------

def test_constant_image_leaves_pose_at_prior(tiny):
    cam = tiny["cam"]
    flat = np.full((cam.H, cam.W), 0.4, np.float32)
    o = oracle.Oracle(oracle.config_for_camera(cam, init_inv_depth=0.3))
    o.set_keyframe(flat, tiny["normals_s"])
    out = o.track(flat, 25)
    st = o.get_state()
    assert np.all(st[..., :6] == 0.0) and np.all(out["xi"] == 0.0)
    # depth: fronto-parallel normals (zero targets) + prior at log-depth 0
    assert np.ptp(st[..., 6]) < 1e-10
    assert abs(st[0, 0, 6]) < abs(math.log(1 / 0.3))


def test_decoupled_pixels_take_gauss_newton_steps(tiny):
    # without identity and normal factors every pixel is its own 7-D problem and
    # each iteration is one Gauss-Newton step on photometric + prior terms
    cam = tiny["cam"]
    kw = dict(sigma_R=math.inf, sigma_N=math.inf, huber_k=2.0)
    o = make(tiny, init_inv_depth=0.4, **kw)
    prob = dense.Problem(cam.H, cam.W, K_of(cam), tiny["I_s"], tiny["I_t"], tiny["normals_s"], **kw)
    st0 = o.get_state()
    o.iterate(1)
    st1 = o.get_state()
    for (u, v) in [(0, 0), (7, 3), (31, 23), (16, 12)]:
        i = v * cam.W + u
        tau, ell = st0[v, u, :6], st0[v, u, 6]
        ok, r, J, w = prob.photometric(i, tau, ell)
        rp, Jp = prob.prior(tau, ell)
        Lm = prob.lamP * Jp.T @ Jp + (w * np.outer(J, J) if ok else 0)
        g = prob.lamP * Jp.T @ rp + (w * J * r if ok else 0)
        d = -np.linalg.solve(Lm, g)
        tau_new = dense.log_se3(dense.exp_se3(tau) @ dense.exp_se3(d[:6]))
        np.testing.assert_allclose(st1[v, u, :6], tau_new, atol=1e-12)
        assert abs(st1[v, u, 6] - (ell + d[6])) < 1e-12


def test_mirror_symmetry():
    # mirroring the images about the principal column flips the sign of the
    # x-translation, the yaw and the roll and mirrors the depth map
    H, W = 12, 16
    rv, tr = [0.002, 0.006, -0.003], [0.012, -0.004, 0.006]
    p = synth.tiny_pair(5, H=H, W=W, rotvec=rv, trans=tr, principal=((W - 1) / 2.0, (H - 1) / 2.0))
    cam = p["cam"]
    normals = p["normals_s"]
    nm = normals[:, ::-1].copy()
    nm[..., 0] *= -1
    kw = dict(init_inv_depth=0.4, huber_k=3.0)
    o1 = oracle.Oracle(oracle.config_for_camera(cam, **kw))
    o1.set_keyframe(p["I_s"], normals)
    r1 = o1.track(p["I_t"], 15)
    o2 = oracle.Oracle(oracle.config_for_camera(cam, **kw))
    o2.set_keyframe(p["I_s"][:, ::-1].copy(), nm)
    r2 = o2.track(p["I_t"][:, ::-1].copy(), 15)
    flip = np.array([1, -1, -1, -1, 1, 1])
    np.testing.assert_allclose(r2["xi"], flip * r1["xi"], atol=1e-10)
    np.testing.assert_allclose(r2["inv_depth"], r1["inv_depth"][:, ::-1], rtol=1e-9)
    assert np.abs(r1["xi"]).max() > 1e-4


def test_full_lie_jacobians_coincide_at_consensus(tiny):
    # with all pixel poses equal the identity residuals vanish and the exact
    # Lie Jacobians reduce to +-I
    outs = []
    for fj in (0, 1):
        o = make(tiny, init_inv_depth=0.4, full_jacobian=fj)
        st = o.get_state()
        st[..., :6] = [0.01, -0.02, 0.005, 0.03, 0.01, -0.02]
        o.set_state(st)
        o.iterate(1)
        outs.append(o.get_state())
    np.testing.assert_allclose(outs[0], outs[1], rtol=1e-10, atol=1e-6)


# --- per-frame outputs -----------------------------------------------------------------

def test_estimator_outputs_and_flags(tiny):
    cam = tiny["cam"]
    o = make(tiny, init_inv_depth=0.3, kf_max_frames=3)
    outs = [o.track(tiny["I_t"], 5) for _ in range(3)]
    st = o.get_state()
    # pose = arithmetic mean of the per-pixel poses (Eq. estimator_avg)
    np.testing.assert_allclose(outs[-1]["xi"], st[..., :6].reshape(-1, 6).mean(0), rtol=1e-14, atol=1e-18)
    np.testing.assert_allclose(outs[-1]["inv_depth"], np.exp(-st[..., 6]), rtol=1e-15)
    lam, _ = o.beliefs()
    var = np.linalg.inv(lam.reshape(-1, 7, 7))[:, 6, 6].reshape(cam.H, cam.W)
    np.testing.assert_allclose(outs[-1]["inv_depth_var"], np.exp(-2 * st[..., 6]) * var, rtol=1e-10)
    assert [r["frames_since_keyframe"] for r in outs] == [1, 2, 3]
    assert [r["flags"] & oracle.KEYFRAME_DUE for r in outs] == [0, 0, oracle.KEYFRAME_DUE]
    assert 0.5 < outs[0]["valid_fraction"] <= 1.0
    # world pose: T_world = T_world_kf Exp(xi)^-1, re-anchoring composes
    np.testing.assert_allclose(outs[-1]["T_world"], np.linalg.inv(oracle.se3_exp(outs[-1]["xi"])), atol=1e-15)
    o.set_keyframe(tiny["I_t"], tiny["normals_s"])
    st2 = o.get_state()
    assert np.all(st2[..., :6] == 0) and np.all(st2[..., 7:] == 0)
    np.testing.assert_array_equal(st2[..., 6], st[..., 6])            # log-depth kept
    r = o.track(tiny["I_t"], 0)
    assert r["frames_since_keyframe"] == 1
    assert r["valid_fraction"] == 1.0          # identity warps stay inside the image
    np.testing.assert_allclose(r["T_world"], outs[-1]["T_world"], atol=1e-15)
    assert np.all(np.isnan(r["inv_depth_var"]))


def test_low_overlap_flag(tiny):
    o = make(tiny, kf_min_valid_frac=0.5)
    st = o.get_state()
    st[..., 3] = 3.0            # 3 m sideways: nothing overlaps
    o.set_state(st)
    r = o.track(tiny["I_t"], 1)
    assert r["valid_fraction"] < 0.5
    assert r["flags"] & oracle.LOW_OVERLAP and r["flags"] & oracle.KEYFRAME_DUE


def test_state_roundtrip(tiny):
    o = make(tiny)
    o.iterate(3)
    s = o.get_state()
    o2 = make(tiny)
    o2.set_state(s)
    np.testing.assert_array_equal(o2.get_state(), s)
    o.iterate(2)
    o2.iterate(2)
    np.testing.assert_array_equal(o2.get_state(), o.get_state())


# --- temporal priors: prior means from the previous estimates ----------------------

def test_frozen_gbp_with_prior_means_equals_dense_solve():
    # a non-identity prior pose mean and a per-pixel log-depth prior map
    p = synth.tiny_pair(4, H=5, W=6, lattice_px=2.0)
    cam = p["cam"]
    kw = dict(sigma_P=1e-2, sigma_R=1e-2, sigma_N=1e-2)
    o = make(p, init_inv_depth=0.4, frozen=1, **kw)
    rng = np.random.default_rng(9)
    xi_hat = rng.normal(0, 0.004, 6)
    ell_hat = np.log(2.5) + rng.normal(0, 0.1, (cam.H, cam.W))
    o.set_prior(xi_hat, ell_hat)
    st = o.get_state()
    st[..., :6] = rng.normal(0, 0.003, size=st[..., :6].shape)
    o.set_state(st)
    prob = dense.Problem(cam.H, cam.W, K_of(cam), p["I_s"], p["I_t"], p["normals_s"], prior_xi=xi_hat,
                         prior_log_depth=ell_hat, **kw)
    ref = prob.solve_linear(st[..., :6].reshape(-1, 6), st[..., 6].reshape(-1))
    o.iterate(400)
    np.testing.assert_allclose(o.means().reshape(-1, 7), ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_prior_from_state_takes_the_current_estimates():
    p = synth.tiny_pair(0)
    o = make(p, init_inv_depth=0.3, sigma_P=0.1)
    o.iterate(5)
    st = o.get_state()
    o.set_prior_from_state()
    # at the prior means the prior residual vanishes: a pixel whose pose equals
    # the mean pose and whose log-depth is its own prior gets no prior gradient
    xi_bar = st[..., :6].reshape(-1, 6).mean(0)
    st2 = st.copy()
    st2[..., :6] = xi_bar
    o.set_state(st2)
    eta, lam, _ = o.unary(3, 4)
    o2 = make(p, init_inv_depth=0.3, sigma_P=np.inf)
    o2.set_state(st2)
    eta2, lam2, _ = o2.unary(3, 4)
    np.testing.assert_allclose(eta, eta2, atol=1e-9 * max(1.0, np.abs(eta2).max()))
