"""Pins of the centralised IRLS Gauss-Newton reference (oracle/centralised.py,
Sec. 3.1 and the centralised baseline of Sec. 4.4): its normal equations are
the per-pixel model's (oracle/dense.py) projected onto exact consensus, with
the N per-pixel pose priors replaced by one, the
true motion and depth of a zero-residual scene are a fixed point, IRLS
converges there from the standard start, and a converged point is stationary
for the nonlinear energy."""

import math

import numpy as np
import pytest

import oracle
import synth
from oracle import dense
from oracle.centralised import Centralised


def K_of(cam):
    return (cam.fx, cam.fy, cam.cx, cam.cy)


def consensus_projection(N):
    """P maps [d_xi; d_ell] to the per-pixel variables (every pixel's pose
    step is d_xi)."""
    P = np.zeros((7 * N, 6 + N))
    for i in range(N):
        P[7 * i:7 * i + 6, :6] = np.eye(6)
        P[7 * i + 6, 6 + i] = 1.0
    return P


@pytest.mark.parametrize("huber_k", [400.0, 0.5])
def test_normal_equations_are_the_consensus_projection(huber_k):
    p = synth.tiny_pair(3, H=5, W=6, lattice_px=2.0)
    cam = p["cam"]
    kw = dict(sigma_P=0.1, sigma_N=1e-2, sigma_D=2e-2, huber_k=huber_k)
    rng = np.random.default_rng(1)
    xi = rng.normal(0, 0.01, 6)
    ell = math.log(2.0) + rng.normal(0, 0.1, cam.H * cam.W)
    prior = rng.normal(0, 0.01, 6)
    c = Centralised(cam.H, cam.W, K_of(cam), p["I_s"], p["normals_s"], prior_xi=prior, prior_log_depth=0.3, **kw)
    c.set_frame(p["I_t"])
    M, g, nv = c.normal_equations(xi, ell)
    prob = dense.Problem(cam.H, cam.W, K_of(cam), p["I_s"], p["I_t"], p["normals_s"], sigma_R=float("inf"),
                         prior_xi=prior, prior_log_depth=0.3, **kw)
    N = cam.H * cam.W
    L, h, nv2 = prob.assemble(np.tile(xi, (N, 1)), ell)
    P = consensus_projection(N)
    assert nv == nv2 and 0 < nv < N
    Md = M.toarray()
    # the projection carries N copies of the pose prior; the centralised
    # model keeps one
    rp = dense.log_se3(np.linalg.inv(dense.exp_se3(prior)) @ dense.exp_se3(xi))
    Jp = dense.prior_jac(rp)
    lamP = 0.1 ** -2
    ref_M = P.T @ L @ P
    ref_M[:6, :6] -= (N - 1) * lamP * Jp.T @ Jp
    ref_g = P.T @ h
    ref_g[:6] += (N - 1) * lamP * Jp.T @ rp
    np.testing.assert_allclose(Md, ref_M, rtol=0, atol=1e-9 * np.abs(Md).max())
    np.testing.assert_allclose(g, ref_g, rtol=0, atol=1e-9 * np.abs(g).max())
    np.testing.assert_array_equal(Md, Md.T)
    if huber_k < 1:
        # the weighting is active somewhere
        valid, r, J, w = c.photometric(xi, ell)
        assert np.any(w[valid] < np.max(w[valid]) * 0.999)


def _zero_residual(p):
    cam = p["cam"]
    tau_true = oracle.se3_log(p["T_ts"])
    ell_true = np.full((cam.H, cam.W), math.log(2.0))
    I_s0 = dense.zero_residual_source(p["I_t"], K_of(cam), tau_true, ell_true, p["I_s"])
    return tau_true, I_s0


def test_truth_is_a_fixed_point_and_irls_converges_to_it():
    p = synth.tiny_pair(0)
    cam = p["cam"]
    tau_true, I_s0 = _zero_residual(p)
    c = Centralised(cam.H, cam.W, K_of(cam), I_s0, p["normals_s"], sigma_P=0.01, prior_xi=tau_true,
                    prior_log_depth=math.log(2.0))
    c.set_frame(p["I_t"])
    dx, dl = c.step(tau_true, np.full(cam.H * cam.W, math.log(2.0)))
    assert np.abs(dx).max() < 1e-12 and np.abs(dl).max() < 1e-12
    xi, ell = c.iterate(np.zeros(6), np.full(cam.H * cam.W, -math.log(0.3)), 15)
    assert np.abs(xi - tau_true).max() < 1e-8
    assert np.abs(np.exp(-ell) - 0.5).max() < 1e-8


def test_irls_reaches_a_fixed_point_that_lowers_the_energy():
    # from the standard start IRLS reaches a point where the Gauss-Newton
    # step vanishes (the right-hand side -J^T Lambda r is zero with the
    # method's Jacobians: image-gradient photometric rows and the truncated
    # prior Jacobian, so this is not the exact energy's stationary point) and
    # the energy there is far below the start
    # a coarser texture keeps every warp inside the image along the way
    p = synth.tiny_pair(3, H=5, W=6, lattice_px=3.0, rotvec=[0, 0, 0], trans=[0.0, 0.0, -0.1])
    cam = p["cam"]
    kw = dict(sigma_P=0.1, sigma_N=1e-2, sigma_D=2e-2, huber_k=1.0)
    c = Centralised(cam.H, cam.W, K_of(cam), p["I_s"], p["normals_s"], **kw)
    c.set_frame(p["I_t"])
    x0, l0 = np.zeros(6), np.full(30, -math.log(0.4))
    xi, ell = c.iterate(x0, l0, 30)
    M, g, nv = c.normal_equations(xi, ell)
    assert nv == 30 and np.abs(g).max() < 1e-8 * np.abs(M.diagonal()).max()
    dx, dl = c.step(xi, ell)
    assert np.abs(dx).max() < 1e-10 and np.abs(dl).max() < 1e-10

    def energy(x, l):
        valid, r, J, w = c.photometric(x, l)
        Mw = np.abs(r) / c.sigD.reshape(-1)
        E = np.sum(np.where(valid, np.where(Mw <= c.k, 0.5 * Mw * Mw, c.k * Mw - 0.5 * c.k * c.k), 0.0))
        rp = dense.log_se3(np.linalg.inv(dense.exp_se3(c.prior_xi)) @ dense.exp_se3(x))
        E += 0.5 * c.lamP * rp @ rp + 0.5 * c.lamP * np.sum((l - c.prior_ell) ** 2)
        a, b, cc = c.normal_edges()
        return E + 0.5 * c.lamN * np.sum((l[b] - l[a] + cc) ** 2)

    assert energy(xi, ell) < 0.1 * energy(x0, l0)
