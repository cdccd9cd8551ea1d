"""Pins of the oracle's building blocks against definitions it does not share:
scipy's matrix exponential/logarithm, central finite differences, closed forms
of the Huber weight, and covariance-form Gaussian marginalisation."""

import math

import numpy as np
import pytest

import oracle
from oracle import dense

rng = np.random.default_rng(1234)


def rand_xi(scale=0.3):
    return rng.normal(0.0, scale, size=6)


# --- SE(3) -------------------------------------------------------------------

@pytest.mark.parametrize("scale", [1e-9, 1e-5, 1e-3, 0.1, 0.8, 2.5])
def test_exp_matches_matrix_exponential(scale):
    for _ in range(5):
        xi = rand_xi(scale)
        np.testing.assert_allclose(oracle.se3_exp(xi), dense.exp_se3(xi), rtol=0, atol=1e-14 + 1e-13 * scale)


@pytest.mark.parametrize("scale", [1e-9, 1e-5, 1e-3, 0.1, 0.8, 2.0])
def test_log_inverts_exp(scale):
    for _ in range(5):
        xi = rand_xi(scale)
        if np.linalg.norm(xi[:3]) > 3.0:
            continue
        np.testing.assert_allclose(oracle.se3_log(oracle.se3_exp(xi)), xi, rtol=1e-12, atol=1e-15)


def test_log_matches_matrix_logarithm():
    for _ in range(10):
        T = dense.exp_se3(rand_xi(0.5))
        np.testing.assert_allclose(oracle.se3_log(T), dense.log_se3(T), atol=1e-12)


def test_log_near_pi():
    xi = np.array([0.0, 0.0, math.pi - 1e-6, 0.3, -0.2, 0.1])
    T = dense.exp_se3(xi)
    np.testing.assert_allclose(oracle.se3_exp(oracle.se3_log(T)), T, atol=1e-9)


def test_right_jacobian_by_finite_differences():
    # Exp(xi + d) = Exp(xi) Exp(J_r(xi) d) + O(|d|^2)
    for _ in range(5):
        xi = rand_xi(0.4)
        Jr = oracle.se3_jr(xi)
        h = 1e-6
        fd = np.zeros((6, 6))
        for k in range(6):
            e = np.zeros(6)
            e[k] = h
            p = dense.log_se3(np.linalg.inv(dense.exp_se3(xi)) @ dense.exp_se3(xi + e))
            m = dense.log_se3(np.linalg.inv(dense.exp_se3(xi)) @ dense.exp_se3(xi - e))
            fd[:, k] = (p - m) / (2 * h)
        np.testing.assert_allclose(Jr, fd, atol=1e-8)


def test_prior_jacobian_truncation_order():
    # d/dd Log(Exp(xi) Exp(d)) = J_r^-1(xi); the prior Jacobian keeps its series
    # up to ad^2, so the error must scale as |xi|^4.
    errs = []
    for s in [0.2, 0.1, 0.05]:
        xi = np.array([0.3, -0.5, 0.8, 0.2, 0.4, -0.6]) * s
        Jinv = np.linalg.inv(oracle.se3_jr(xi))
        errs.append(np.abs(oracle.prior_jacobian(xi) - Jinv).max())
        np.testing.assert_allclose(oracle.prior_jacobian(xi), dense.prior_jac(xi), atol=1e-15)
    assert errs[0] / errs[1] > 12 and errs[1] / errs[2] > 12      # ~2^4


# --- Huber covariance weighting ------------------------------------------------

def test_huber_weight_closed_form():
    k = 2.0
    for M in [0.0, 0.5, 1.999, 2.0]:
        assert oracle.huber_weight(M, k) == 1.0
    for M in [2.5, 4.0, 100.0]:
        # kappa M^2 / 2 equals the Huber energy k M - k^2/2
        assert abs(oracle.huber_weight(M, k) * M * M / 2 - (k * M - k * k / 2)) < 1e-12 * M * M
    # continuity of kappa and of d kappa / dM at M = k
    eps = 1e-7
    assert abs(oracle.huber_weight(k + eps, k) - 1.0) < 1e-12
    d = (oracle.huber_weight(k + 2 * eps, k) - oracle.huber_weight(k + eps, k)) / eps
    assert abs(d) < 1e-5
    assert oracle.huber_weight(-3.0, k) == oracle.huber_weight(3.0, k)


# --- warp --------------------------------------------------------------------

def test_warp_jacobian_by_finite_differences(tiny):
    cam = tiny["cam"]
    o = oracle.Oracle(oracle.config_for_camera(cam))
    for _ in range(10):
        tau = rand_xi(0.05)
        ell = rng.uniform(-0.5, 1.0)
        u, v = rng.uniform(0, cam.W - 1), rng.uniform(0, cam.H - 1)
        ok, w, J = o.warp(u, v, tau, ell)
        assert ok
        h = 1e-6
        fd = np.zeros((2, 7))
        for k in range(7):
            if k < 6:
                e = np.zeros(6)
                e[k] = h
                tp = oracle.se3_log(oracle.se3_exp(tau) @ oracle.se3_exp(e))
                tm = oracle.se3_log(oracle.se3_exp(tau) @ oracle.se3_exp(-e))
                fd[:, k] = (o.warp(u, v, tp, ell)[1] - o.warp(u, v, tm, ell)[1]) / (2 * h)
            else:
                fd[:, k] = (o.warp(u, v, tau, ell + h)[1] - o.warp(u, v, tau, ell - h)[1]) / (2 * h)
        np.testing.assert_allclose(J, fd, rtol=1e-6, atol=1e-6)
        # the NumPy re-derivation agrees to rounding
        okd, wd, Jd = dense.warp_pixel((cam.fx, cam.fy, cam.cx, cam.cy), u, v, tau, ell)
        np.testing.assert_allclose(w, wd, atol=1e-11)
        np.testing.assert_allclose(J, Jd, rtol=1e-10, atol=1e-10)


def test_identity_warp_is_identity(tiny):
    cam = tiny["cam"]
    o = oracle.Oracle(oracle.config_for_camera(cam))
    for (u, v) in [(0, 0), (cam.W - 1, cam.H - 1), (5, 7)]:
        ok, w, _ = o.warp(u, v, np.zeros(6), 0.7)
        assert ok
        np.testing.assert_allclose(w, [u, v], atol=1e-12)


# --- unary factors -----------------------------------------------------------

def _oracle_on(p, **kw):
    cam = p["cam"]
    o = oracle.Oracle(oracle.config_for_camera(cam, **kw))
    o.set_keyframe(p["I_s"], p["normals_s"])
    o.set_frame(p["I_t"])
    return o


@pytest.mark.parametrize("huber_k", [400.0, 0.5])
def test_unary_matches_dense_rederivation(tiny, huber_k):
    p = tiny
    cam = p["cam"]
    o = _oracle_on(p, huber_k=huber_k, init_inv_depth=0.4)
    st = o.get_state()
    # move the linearisation points off zero so every Jacobian block is exercised
    st[..., :6] = rng.normal(0, 0.01, size=(cam.H, cam.W, 6))
    st[..., 6] += rng.normal(0, 0.1, size=(cam.H, cam.W))
    o.set_state(st)
    prob = dense.Problem(cam.H, cam.W, (cam.fx, cam.fy, cam.cx, cam.cy), p["I_s"], p["I_t"], p["normals_s"],
                         huber_k=huber_k)
    for (u, v) in [(0, 0), (3, 4), (cam.W - 1, cam.H - 1), (17, 11)]:
        eta, lam, valid = o.unary(u, v)
        i = v * cam.W + u
        tau, ell = st[v, u, :6], st[v, u, 6]
        ok, r, J, wgt = prob.photometric(i, tau, ell)
        rp, Jp = prob.prior(tau, ell)
        lam_ref = prob.lamP * Jp.T @ Jp + (wgt * np.outer(J, J) if ok else 0)
        eta_ref = -prob.lamP * Jp.T @ rp - (wgt * J * r if ok else 0)
        assert valid == ok
        np.testing.assert_allclose(lam, lam_ref, rtol=1e-9, atol=1e-9 * np.abs(lam_ref).max())
        np.testing.assert_allclose(eta, eta_ref, rtol=1e-9, atol=1e-9 * np.abs(eta_ref).max())


def test_gradient_images(tiny):
    o = _oracle_on(tiny)
    gx, gy = o.gradients()
    I = tiny["I_t"].astype(np.float64)
    assert gx[5, 7] == 0.5 * (I[5, 8] - I[5, 6])
    assert gx[5, 0] == I[5, 1] - I[5, 0]
    assert gy[0, 3] == I[1, 3] - I[0, 3]
    assert gy[-1, 3] == I[-1, 3] - I[-2, 3]
    # a linear ramp has the exact gradient everywhere, borders included
    ramp = (0.01 * np.arange(32)[None, :] + 0.02 * np.arange(24)[:, None]).astype(np.float32)
    o.set_frame(ramp)
    gx, gy = o.gradients()
    np.testing.assert_allclose(gx, 0.01, atol=1e-6)
    np.testing.assert_allclose(gy, 0.02, atol=1e-6)


def test_pure_rotation_has_no_depth_information(tiny):
    # with zero translation the warp does not depend on depth: J_logdepth = 0
    o = _oracle_on(tiny)
    st = o.get_state()
    st[..., :3] = [0.002, -0.004, 0.001]
    st[..., 3:6] = 0.0
    o.set_state(st)
    eta, lam, valid = o.unary(10, 10)
    assert valid
    lamP = 1.0
    assert abs(lam[6, 6] - lamP) < 1e-12 and np.abs(lam[6, :6]).max() < 1e-12


def test_normal_targets_of_planes():
    # a plane n.X = d imaged by the pinhole camera has log-depth
    # ell(u,v) = log d - log(n.q(u,v)); the normal-integration residual
    # (ell_b - ell_a) + c_a is the first-order Taylor remainder, O(c^2)
    H, W = 12, 16
    K = (20.0, 22.0, 7.5, 6.0)
    n = np.array([0.3, -0.2, -0.93])
    n /= np.linalg.norm(n)
    normals = np.broadcast_to(n.astype(np.float32), (H, W, 3)).copy()
    cfg = oracle.default_config(H=H, W=W, fx=K[0], fy=K[1], cx=K[2], cy=K[3])
    o = oracle.Oracle(cfg)
    o.set_keyframe(np.zeros((H, W), np.float32), normals)
    cxt, cyt = o.normal_targets()
    u, v = np.meshgrid(np.arange(W), np.arange(H))
    q = np.stack([(u - K[2]) / K[0], (v - K[3]) / K[1], np.ones_like(u, dtype=float)], -1)
    ell = np.log(-2.0) if False else -np.log(np.abs(q @ n.astype(np.float32).astype(np.float64)))
    rx = ell[:, 1:] - ell[:, :-1] + cxt[:, :-1]
    ry = ell[1:, :] - ell[:-1, :] + cyt[:-1, :]
    assert np.abs(rx).max() < 2 * np.nanmax(np.abs(cxt)) ** 2
    assert np.abs(ry).max() < 2 * np.nanmax(np.abs(cyt)) ** 2
    # fronto-parallel: zero targets
    o.set_keyframe(np.zeros((H, W), np.float32), np.broadcast_to(np.float32([0, 0, -1]), (H, W, 3)).copy())
    cxt, cyt = o.normal_targets()
    assert np.all(cxt == 0) and np.all(cyt == 0)
    # grazing normals deactivate the edge
    g = np.broadcast_to(np.float32([0, 0, -1]), (H, W, 3)).copy()
    g[2, 3] = [1.0, 0.0, 0.0]     # n.q = q_x = (3 - 7.5)/20 != 0 -> active
    g[2, 7] = [1.0, 0.0, 0.0]     # q_x = (7 - 7.5)/20 = -0.025 < 1e-3 |q|? no: active
    g[4, 5] = [0.0, 0.0, 0.0]     # degenerate normal -> inactive
    o.set_keyframe(np.zeros((H, W), np.float32), g)
    cxt, cyt = o.normal_targets()
    assert np.isnan(cxt[4, 5]) and np.isnan(cyt[4, 5])


# --- factor-to-variable messages -------------------------------------------------

def _random_spd(n, scale=1.0):
    A = rng.normal(size=(n, n))
    return scale * (A @ A.T + n * np.eye(n))


def test_identity_message_equals_covariance_form_marginal():
    lamR = 50.0
    r = rng.normal(0, 0.1, size=6)
    J = np.zeros((6, 14))
    J[:, :6] = np.eye(6)
    J[:, 7:13] = -np.eye(6)
    lam_s = _random_spd(7)
    eta_s = rng.normal(size=7)
    eta, lam = oracle.factor_message(r, J, [lamR] * 6, eta_s, lam_s)
    Lf = J.T @ (lamR * J)
    hf = -J.T @ (lamR * r)
    eta_ref, lam_ref = dense.marginal_message_covariance_form(Lf, hf, lam_s, eta_s, 3.0 * np.eye(7))
    np.testing.assert_allclose(lam, lam_ref, atol=1e-9)
    np.testing.assert_allclose(eta, eta_ref, atol=1e-9)
    # the factor does not touch the receiver's depth
    assert np.all(lam[6, :] == 0) and np.all(lam[:, 6] == 0) and eta[6] == 0
    # series-combination form: Lambda' = lamR (lamR I + P)^-1 P with P the
    # sender's pose marginal
    P = lam_s[:6, :6] - np.outer(lam_s[:6, 6], lam_s[6, :6]) / lam_s[6, 6]
    np.testing.assert_allclose(lam[:6, :6], lamR * np.linalg.solve(lamR * np.eye(6) + P, P), atol=1e-9)


def test_normal_message_closed_form():
    lamN = 7.0
    lam_s = _random_spd(7)
    eta_s = rng.normal(size=7)
    c = 0.03
    ell_a, ell_b = 0.2, 0.35
    rn = ell_b - ell_a + c
    # depth marginal of the sender's message
    S = lam_s[:6, :6]
    lam_d = lam_s[6, 6] - lam_s[6, :6] @ np.linalg.solve(S, lam_s[:6, 6])
    eta_d = eta_s[6] - lam_s[6, :6] @ np.linalg.solve(S, eta_s[:6])
    for recv_is_b in (True, False):
        J = np.zeros(14)
        J[6] = 1.0 if recv_is_b else -1.0
        J[13] = -J[6]
        eta, lam = oracle.factor_message([rn], J, [lamN], eta_s, lam_s)
        assert abs(lam[6, 6] - lamN * lam_d / (lamN + lam_d)) < 1e-12
        sgn = 1.0 if recv_is_b else -1.0
        eta_ref = lamN * (eta_d - sgn * lam_d * rn) / (lamN + lam_d)
        assert abs(eta[6] - eta_ref) < 1e-12
        assert np.all(lam[:6, :] == 0) and np.all(eta[:6] == 0)
