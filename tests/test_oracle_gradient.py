"""Pins of the oracle's gradient (central differences of unrolled tracking,
oracle/gradient.py) against an independent derivative.

At a converged fixed point of relinearised GBP (equal to the dense
Gauss-Newton / IRLS fixed point, pinned in test_oracle_gbp.py), the model's
gradient vanishes: F(delta, theta) = h(x* (+) delta; theta) = 0, with h the
right-hand side of the dense normal equations (oracle/dense.py, NumPy,
scipy's matrix exponential and logarithm). The implicit function theorem
gives the fixed point's derivative d delta / d theta = -(dF/d delta)^-1
dF/d theta, both Jacobians taken by differences of the dense assembly. Pushed
through the outputs (pose mean, inverse depth), this is the exact derivative
of the converged oracle, which the oracle's finite differences must match.
"""

import numpy as np
import pytest

import synth
from oracle import Oracle, config_for_camera, dense
from oracle.gradient import UnrolledOracle, central_difference, relative_sensitivity


def K_of(cam):
    return (cam.fx, cam.fy, cam.cx, cam.cy)


N_ITERS = 4000     # the difference quotients converge more slowly than the means
STEP = 1e-5


def _setup(huber_k):
    # backward motion keeps every warp inside the image (no valid-set changes);
    # pixel noise leaves residuals at the fixed point, so a small threshold
    # makes the Huber weighting active
    p = synth.tiny_pair(3, H=4, W=5, lattice_px=2.0, rotvec=[0, 0, 0], trans=[0.0, 0.0, -0.05])
    p["I_t"] = (p["I_t"] + np.random.default_rng(5).normal(0.0, 0.003, p["I_t"].shape)).astype(np.float32)
    cam = p["cam"]
    sig = np.full((cam.H, cam.W), 2e-2) * (1.0 + 0.1 * np.random.default_rng(1).uniform(-1, 1, (cam.H, cam.W)))
    kw = dict(sigma_P=1e-1, sigma_R=1e-2, init_inv_depth=0.4)
    uo = UnrolledOracle(cam, p["I_s"], p["normals_s"], [p["I_t"]], N_ITERS, sig, 1e-2, huber_k, **kw)
    rng = np.random.default_rng(2)
    cxi = rng.normal(size=(1, 6))
    crho = rng.normal(size=(1, cam.H, cam.W))
    return p, cam, sig, uo, cxi, crho


def _implicit_derivatives(p, cam, sig, huber_k, cxi, crho, entry):
    """Derivatives of the functional at the converged outputs with respect to
    sigma_N, huber_k and sigma_D[entry], by the implicit function theorem on
    the dense model."""
    N = cam.H * cam.W

    def problem(sigma_N=1e-2, k=huber_k, smap=sig):
        return dense.Problem(cam.H, cam.W, K_of(cam), p["I_s"], p["I_t"], p["normals_s"], sigma_D_map=smap,
                             sigma_P=1e-1, sigma_R=1e-2, sigma_N=sigma_N, huber_k=k)

    # the fixed point: a few dense Gauss-Newton steps from the oracle's
    # converged state (the characterisation h = 0 is the dense model's)
    o = Oracle(config_for_camera(cam, sigma_P=1e-1, sigma_R=1e-2, sigma_N=1e-2, huber_k=huber_k, init_inv_depth=0.4))
    o.set_sigma_D_map(sig)
    o.set_keyframe(p["I_s"], p["normals_s"])
    o.set_frame(p["I_t"])
    o.iterate(N_ITERS)
    st = o.get_state()
    o.close()
    prob = problem()
    tau, ell = prob.gauss_newton(st[..., :6].reshape(-1, 6), st[..., 6].reshape(-1), 3)
    assert np.abs(prob.assemble(tau, ell)[1]).max() < 1e-6
    assert np.abs(tau - st[..., :6].reshape(-1, 6)).max() < 1e-7

    def F(delta):
        t2 = np.array([dense.log_se3(dense.exp_se3(tau[i]) @ dense.exp_se3(delta[7 * i:7 * i + 6]))
                       for i in range(N)])
        return prob.assemble(t2, ell + delta[6::7])[1]

    n = 7 * N
    A = np.zeros((n, n))
    hd = 1e-6
    for j in range(n):
        d = np.zeros(n)
        d[j] = hd
        A[:, j] = (F(d) - F(-d)) / (2 * hd)
    ht = 1e-6
    v, u = entry
    mp, mm = sig.copy(), sig.copy()
    mp[v, u] *= 1 + ht
    mm[v, u] *= 1 - ht
    bs = {
        "sigma_N": (problem(sigma_N=1e-2 * (1 + ht)).assemble(tau, ell)[1] -
                    problem(sigma_N=1e-2 * (1 - ht)).assemble(tau, ell)[1]) / (2 * ht * 1e-2),
        "huber_k": (problem(k=huber_k * (1 + ht)).assemble(tau, ell)[1] -
                    problem(k=huber_k * (1 - ht)).assemble(tau, ell)[1]) / (2 * ht * huber_k),
        "sigma_D": (problem(smap=mp).assemble(tau, ell)[1] - problem(smap=mm).assemble(tau, ell)[1]) /
                   (2 * ht * sig[v, u]),
    }
    # outputs: tau_i (+) delta_i gives d tau_i = Jr(tau_i)^-1 d delta_i (by
    # differences of the dense Exp/Log); rho_i = exp(-ell_i)
    Jinv = []
    for i in range(N):
        Ji = np.zeros((6, 6))
        for j in range(6):
            e = np.zeros(6)
            e[j] = 1e-6
            Ji[:, j] = (dense.log_se3(dense.exp_se3(tau[i]) @ dense.exp_se3(e)) -
                        dense.log_se3(dense.exp_se3(tau[i]) @ dense.exp_se3(-e))) / 2e-6
        Jinv.append(Ji)
    out = {}
    for name, b in bs.items():
        dd = -np.linalg.solve(A, b)
        dxi = sum(Jinv[i] @ dd[7 * i:7 * i + 6] for i in range(N)) / N
        drho = -np.exp(-ell) * dd[6::7]
        out[name] = float(np.sum(cxi[0] * dxi) + np.sum(crho[0].reshape(-1) * drho))
    return out


@pytest.mark.parametrize("huber_k", [400.0, 0.05])
def test_oracle_differences_equal_implicit_derivative(huber_k):
    p, cam, sig, uo, cxi, crho = _setup(huber_k)
    ref = _implicit_derivatives(p, cam, sig, huber_k, cxi, crho, (1, 2))
    fd = {"sigma_N": uo.d_sigma_N(cxi, crho, h=STEP), "sigma_D": uo.d_sigma_entry(cxi, crho, 1, 2, h=STEP)}
    if huber_k < 10:
        fd["huber_k"] = uo.d_huber_k(cxi, crho, h=STEP)
        assert abs(ref["huber_k"]) > 1e-6 * abs(ref["sigma_N"])    # the weighting is active
    for name, g in fd.items():
        print(f"k={huber_k} {name}: oracle differences {g:.9e}, implicit {ref[name]:.9e}")
        assert abs(g - ref[name]) <= 1e-4 * abs(ref[name])


def test_difference_helpers_on_closed_forms():
    # central differences are exact for quadratics; the relative-step
    # sensitivity of a smooth function is at the difference quotient's
    # truncation level
    f = lambda x: 3.0 * x * x - 2.0 * x + 1.0
    assert abs(central_difference(f, 0.7, 1e-3) - (6.0 * 0.7 - 2.0)) < 1e-9
    assert relative_sensitivity(np.exp, 1.3) < 1e-8
