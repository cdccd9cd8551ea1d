"""Dense NumPy validators for the oracle (test infrastructure only).

Independent of the C oracle: the factor definitions are re-derived here in
vectorised NumPy and assembled into the joint 7N-dimensional problem, so that
the oracle's message passing can be checked against

* the dense normal-equation solve of the linearised model (loopy Gaussian BP
  means, when converged, equal the exact solution);
* a dense Gauss-Newton / IRLS iteration of the nonlinear model (the paper's
  centralised baseline form, Sec. 3.1 and Sec. 4.4), whose fixed point is the
  fixed point of relinearised GBP;
* covariance-form marginalisation of a single factor (Sec. 3.4).

SE(3) here uses scipy's matrix exponential and logarithm of the 4x4 twist
matrix, which is the plain definition of the group exponential.
"""

from __future__ import annotations

import math
from typing import Dict, Optional, Tuple

import numpy as np
import scipy.linalg as sla

WARP_EPS = 1e-3


def hat(xi: np.ndarray) -> np.ndarray:
    w, r = xi[:3], xi[3:]
    X = np.zeros((4, 4))
    X[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    X[:3, 3] = r
    return X


def exp_se3(xi) -> np.ndarray:
    return sla.expm(hat(np.asarray(xi, dtype=np.float64)))


def log_se3(T) -> np.ndarray:
    L = np.real(sla.logm(np.asarray(T, dtype=np.float64)))
    return np.array([L[2, 1], L[0, 2], L[1, 0], L[0, 3], L[1, 3], L[2, 3]])


def ad_se3(xi) -> np.ndarray:
    w, r = xi[:3], xi[3:]
    sw = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    sr = np.array([[0, -r[2], r[1]], [r[2], 0, -r[0]], [-r[1], r[0], 0]])
    A = np.zeros((6, 6))
    A[:3, :3] = sw
    A[3:, :3] = sr
    A[3:, 3:] = sw
    return A


def prior_jac(xi) -> np.ndarray:
    A = ad_se3(xi)
    return np.eye(6) + 0.5 * A + A @ A / 12.0


def huber_kappa(M: np.ndarray, k: float) -> np.ndarray:
    M = np.abs(M)
    with np.errstate(divide="ignore", invalid="ignore"):
        out = np.where(M <= k, 1.0, 2.0 * k / M - (k * k) / (M * M))
    return out


def gradients(I: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    I = I.astype(np.float64)
    gx = np.empty_like(I)
    gy = np.empty_like(I)
    gx[:, 1:-1] = 0.5 * (I[:, 2:] - I[:, :-2])
    gx[:, 0] = I[:, 1] - I[:, 0]
    gx[:, -1] = I[:, -1] - I[:, -2]
    if I.shape[0] == 1:
        gy[:] = 0.0
    else:
        gy[1:-1, :] = 0.5 * (I[2:, :] - I[:-2, :])
        gy[0, :] = I[1, :] - I[0, :]
        gy[-1, :] = I[-1, :] - I[-2, :]
    return gx, gy


def bilinear(img: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    H, W = img.shape
    if H == 1:
        x0 = np.clip(np.floor(x).astype(np.int64), 0, W - 2)
        fx = x - x0
        I = img.astype(np.float64)[0]
        return (1 - fx) * I[x0] + fx * I[x0 + 1]
    x0 = np.clip(np.floor(x).astype(np.int64), 0, W - 2)
    y0 = np.clip(np.floor(y).astype(np.int64), 0, H - 2)
    fx, fy = x - x0, y - y0
    I = img.astype(np.float64)
    return ((1 - fy) * ((1 - fx) * I[y0, x0] + fx * I[y0, x0 + 1])
            + fy * ((1 - fx) * I[y0 + 1, x0] + fx * I[y0 + 1, x0 + 1]))


def normal_targets(normals: np.ndarray, K) -> Tuple[np.ndarray, np.ndarray]:
    fx, fy, cx, cy = K
    H, W, _ = normals.shape
    u, v = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    q = np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u)], -1)
    n = normals.astype(np.float64)
    nq = np.sum(n * q, -1)
    ok = np.isfinite(nq) & (np.abs(nq) >= 1e-3 * np.linalg.norm(q, axis=-1))
    with np.errstate(divide="ignore", invalid="ignore"):
        cxt = np.where(ok, n[..., 0] / (fx * nq), np.nan)
        cyt = np.where(ok, n[..., 1] / (fy * nq), np.nan)
    return cxt, cyt


def warp_pixel(K, u: float, v: float, tau, ell: float):
    """w(tau, ell) for pixel (u, v) and the 2x7 Jacobian with respect to a
    right perturbation of the pose and an additive log-depth step."""
    fx, fy, cx, cy = K
    T = exp_se3(tau)
    R, t = T[:3, :3], T[:3, 3]
    q = np.array([(u - cx) / fx, (v - cy) / fy, 1.0])
    rho = math.exp(-ell)
    a = R @ q + rho * t
    w = np.array([fx * a[0] / a[2] + cx, fy * a[1] / a[2] + cy])
    dwda = np.array([[fx / a[2], 0, -fx * a[0] / a[2] ** 2], [0, fy / a[2], -fy * a[1] / a[2] ** 2]])
    qx = np.array([[0, -q[2], q[1]], [q[2], 0, -q[0]], [-q[1], q[0], 0]])
    dadx = np.zeros((3, 7))
    dadx[:, :3] = -R @ qx
    dadx[:, 3:6] = rho * R
    dadx[:, 6] = -rho * t
    return a[2] > 0, w, dwda @ dadx


def quadtree_levels(H: int, W: int):
    """Level sizes [(rows, cols)] of the quadtree of pose variables (Fig. 2,
    Sec. 4.2): level 0 is the H x W pixel array, level l has ceil(H / 2^l) x
    ceil(W / 2^l) nodes, each joined to the 2 x 2 block below it, up to the
    single root."""
    dims = [(H, W)]
    l = 0
    while dims[-1] != (1, 1):
        l += 1
        dims.append((-(-H // 2 ** l), -(-W // 2 ** l)))
    return dims


def level_sigmas(sigma: float, n_levels: int):
    """sigma halved at each level above the leaves (Sec. 4.2)."""
    return [sigma * 0.5 ** l for l in range(n_levels)]


class Problem:
    """The linearisable model of one keyframe / target-frame pair on an H x W grid.

    topology "grid": identity factors between 4-neighbour pixels (Eq. regul).
    topology "quadtree": identity factors only between each variable and its
    parent in the quadtree (pixels at level 0, 6-D pose nodes above); the
    prior and identity sigmas halve per level (Sec. 4.2), the identity factor
    between levels l and l + 1 taking the level-l value. Node variables follow
    the 7N pixel variables, 6 per node, level-major and row-major."""

    def __init__(self, H, W, K, I_s, I_t, normals, sigma_D=5e-3, sigma_P=1.0, sigma_R=4e-4,
                 sigma_N=1e-3, huber_k=400.0, prior_xi=None, prior_log_depth=0.0, sigma_D_map=None,
                 topology="grid"):
        assert topology in ("grid", "quadtree")
        self.topology = topology
        self.levels = quadtree_levels(H, W) if topology == "quadtree" else [(H, W)]
        self.sigma_P, self.sigma_R = sigma_P, sigma_R
        offs = [0, 0]
        for (h, w) in self.levels[1:]:
            offs.append(offs[-1] + h * w)
        self.level_offset = offs        # first node of level l >= 1
        self.NT = offs[-1]
        self.H, self.W, self.K = H, W, tuple(float(k) for k in K)
        self.I_s = I_s.astype(np.float64)
        self.I_t = I_t.astype(np.float64)
        self.Gx, self.Gy = gradients(I_t)
        self.cxt, self.cyt = normal_targets(normals, self.K)
        self.sigD = np.full((H, W), sigma_D) if sigma_D_map is None else np.asarray(sigma_D_map, dtype=np.float64)
        self.lamP = sigma_P ** -2
        self.lamR = 0.0 if math.isinf(sigma_R) else sigma_R ** -2
        self.lamN = 0.0 if math.isinf(sigma_N) else sigma_N ** -2
        self.k = huber_k
        self.prior_xi = np.zeros(6) if prior_xi is None else np.asarray(prior_xi, dtype=np.float64)
        # scalar or per-pixel (H x W) log-depth prior mean
        self.prior_ell = np.broadcast_to(np.asarray(prior_log_depth, dtype=np.float64), (H, W)).reshape(-1)

    @property
    def N(self):
        return self.H * self.W

    def photometric(self, i: int, tau, ell):
        """(valid, residual, 1x7 Jacobian, weight kappa*Lambda_D) of pixel i."""
        u, v = i % self.W, i // self.W
        ok, w, Jw = warp_pixel(self.K, u, v, tau, ell)
        if not ok or not (-WARP_EPS <= w[0] <= self.W - 1 + WARP_EPS and -WARP_EPS <= w[1] <= self.H - 1 + WARP_EPS):
            return False, 0.0, np.zeros(7), 0.0
        x = min(max(w[0], 0.0), self.W - 1.0)
        y = min(max(w[1], 0.0), self.H - 1.0)
        xs, ys = np.array([x]), np.array([y])
        r = self.I_s.flat[i] - bilinear(self.I_t, xs, ys)[0]
        g = np.array([bilinear(self.Gx, xs, ys)[0], bilinear(self.Gy, xs, ys)[0]])
        J = -(g @ Jw)
        lamD = self.sigD.flat[i] ** -2
        kap = huber_kappa(abs(r) * math.sqrt(lamD), self.k)
        return True, r, J, float(kap * lamD)

    def prior(self, tau, ell, i: int = 0):
        rp = log_se3(np.linalg.inv(exp_se3(self.prior_xi)) @ exp_se3(tau))
        J = np.zeros((7, 7))
        J[:6, :6] = prior_jac(rp)
        J[6, 6] = 1.0
        return np.concatenate([rp, [ell - self.prior_ell[i]]]), J

    def edges(self):
        """Undirected edges (a, b, horizontal) with a the left/upper pixel."""
        out = []
        for v in range(self.H):
            for u in range(self.W):
                i = v * self.W + u
                if u + 1 < self.W:
                    out.append((i, i + 1, True))
                if v + 1 < self.H:
                    out.append((i, i + self.W, False))
        return out

    def node(self, l: int, col: int, row: int) -> int:
        return self.level_offset[l] + row * self.levels[l][1] + col

    def tree_edges(self):
        """(child pose column, parent pose column, child level) of every quadtree edge."""
        out = []
        for l in range(len(self.levels) - 1):
            h, w = self.levels[l]
            for row in range(h):
                for col in range(w):
                    c = 7 * (row * self.W + col) if l == 0 else 7 * self.N + 6 * self.node(l, col, row)
                    p = 7 * self.N + 6 * self.node(l + 1, col // 2, row // 2)
                    out.append((c, p, l))
        return out

    def assemble(self, tau: np.ndarray, ell: np.ndarray, ntau: Optional[np.ndarray] = None):
        """Joint information (Lambda, eta) of the model linearised at (tau, ell)
        (and the quadtree node poses ntau), variables ordered pixel-major, 7 per
        pixel, then 6 per node; eta = -J^T Lambda r."""
        N = self.N
        tree = self.topology == "quadtree"
        n = 7 * N + (6 * self.NT if tree else 0)
        L = np.zeros((n, n))
        h = np.zeros(n)
        nvalid = 0
        for i in range(N):
            s = slice(7 * i, 7 * i + 7)
            ok, r, J, wgt = self.photometric(i, tau[i], ell[i])
            if ok:
                nvalid += 1
                L[s, s] += wgt * np.outer(J, J)
                h[s] -= wgt * J * r
            rp, Jp = self.prior(tau[i], ell[i], i)
            L[s, s] += self.lamP * Jp.T @ Jp
            h[s] -= self.lamP * Jp.T @ rp
        if tree:
            nlev = len(self.levels)
            sP = level_sigmas(self.sigma_P, nlev)
            sR = level_sigmas(self.sigma_R, nlev)
            for k in range(self.NT):
                l = max(i for i in range(1, nlev) if self.level_offset[i] <= k)
                s = slice(7 * N + 6 * k, 7 * N + 6 * k + 6)
                rp = log_se3(np.linalg.inv(exp_se3(self.prior_xi)) @ exp_se3(ntau[k]))
                Jp = prior_jac(rp)
                L[s, s] += sP[l] ** -2 * Jp.T @ Jp
                h[s] -= sP[l] ** -2 * Jp.T @ rp
            if self.lamR > 0:
                for (c, p, l) in self.tree_edges():
                    tc = tau[c // 7] if c < 7 * N else ntau[(c - 7 * N) // 6]
                    tp = ntau[(p - 7 * N) // 6]
                    lam = sR[l] ** -2
                    r = log_se3(np.linalg.inv(exp_se3(tp)) @ exp_se3(tc))   # receiver child, sender parent
                    sc, sp = slice(c, c + 6), slice(p, p + 6)
                    L[sc, sc] += lam * np.eye(6)
                    L[sp, sp] += lam * np.eye(6)
                    L[sc, sp] -= lam * np.eye(6)
                    L[sp, sc] -= lam * np.eye(6)
                    h[sc] -= lam * r
                    h[sp] += lam * r
        for (a, b, horiz) in self.edges():
            sa, sb = slice(7 * a, 7 * a + 6), slice(7 * b, 7 * b + 6)
            if self.lamR > 0 and not tree:
                r = log_se3(np.linalg.inv(exp_se3(tau[a])) @ exp_se3(tau[b]))   # receiver b, sender a
                # J_b = +I, J_a = -I
                L[sb, sb] += self.lamR * np.eye(6)
                L[sa, sa] += self.lamR * np.eye(6)
                L[sa, sb] -= self.lamR * np.eye(6)
                L[sb, sa] -= self.lamR * np.eye(6)
                h[sb] -= self.lamR * r
                h[sa] += self.lamR * r
            c = self.cxt.flat[a] if horiz else self.cyt.flat[a]
            if self.lamN > 0 and np.isfinite(c):
                ia, ib = 7 * a + 6, 7 * b + 6
                rn = ell[b] - ell[a] + c
                L[ib, ib] += self.lamN
                L[ia, ia] += self.lamN
                L[ia, ib] -= self.lamN
                L[ib, ia] -= self.lamN
                h[ib] -= self.lamN * rn
                h[ia] += self.lamN * rn
        return L, h, nvalid

    def solve_linear(self, tau, ell):
        L, h, _ = self.assemble(tau, ell)
        return np.linalg.solve(L, h).reshape(self.N, 7)

    def solve_tree(self, tau, ell, ntau):
        """Linear solve of the quadtree model: (pixel steps (N, 7), node steps (NT, 6))."""
        L, h, _ = self.assemble(tau, ell, ntau)
        d = np.linalg.solve(L, h)
        return d[:7 * self.N].reshape(self.N, 7), d[7 * self.N:].reshape(self.NT, 6)

    def gauss_newton_tree(self, tau, ell, ntau, n_iters: int):
        tau = np.array(tau, dtype=np.float64).copy()
        ell = np.array(ell, dtype=np.float64).copy()
        ntau = np.array(ntau, dtype=np.float64).copy()
        for _ in range(n_iters):
            dp, dn = self.solve_tree(tau, ell, ntau)
            for i in range(self.N):
                tau[i] = log_se3(exp_se3(tau[i]) @ exp_se3(dp[i, :6]))
            for k in range(self.NT):
                ntau[k] = log_se3(exp_se3(ntau[k]) @ exp_se3(dn[k]))
            ell = ell + dp[:, 6]
        return tau, ell, ntau

    def gauss_newton(self, tau, ell, n_iters: int, damping: float = 1.0):
        tau = np.array(tau, dtype=np.float64).copy()
        ell = np.array(ell, dtype=np.float64).copy()
        for _ in range(n_iters):
            d = damping * self.solve_linear(tau, ell)
            for i in range(self.N):
                tau[i] = log_se3(exp_se3(tau[i]) @ exp_se3(d[i, :6]))
            ell = ell + d[:, 6]
        return tau, ell


def marginal_message_covariance_form(Lf: np.ndarray, hf: np.ndarray, lam_s: np.ndarray, eta_s: np.ndarray,
                                     lam_0: np.ndarray):
    """Factor-to-variable message computed through covariances.

    The joint over [x_recv; x_send] is the factor (Lf, hf) times the sender's
    variable-to-factor message times an auxiliary prior lam_0 on x_recv (which
    makes the joint proper). The receiver's marginal is read from the joint
    covariance; the message is that marginal with the auxiliary prior removed.
    """
    L = Lf.copy()
    h = hf.copy()
    L[7:, 7:] += lam_s
    h[7:] += eta_s
    L[:7, :7] += lam_0
    S = np.linalg.inv(L)
    mu = S @ h
    Srr = S[:7, :7]
    lam_marg = np.linalg.inv(Srr)
    eta_marg = lam_marg @ mu[:7]
    return eta_marg, lam_marg - lam_0


def zero_residual_source(I_t: np.ndarray, K, tau_true, ell_true: np.ndarray, I_s_fallback: np.ndarray):
    """Source image for which the photometric residual vanishes at (tau_true, ell_true):
    I_s[p] = bilinear(I_t, W(p; tau_true, ell_true)) wherever the warp is valid."""
    H, W = I_t.shape
    out = I_s_fallback.astype(np.float64).copy()
    for v in range(H):
        for u in range(W):
            ok, w, _ = warp_pixel(K, u, v, tau_true, float(ell_true[v, u]))
            if ok and -WARP_EPS <= w[0] <= W - 1 + WARP_EPS and -WARP_EPS <= w[1] <= H - 1 + WARP_EPS:
                x = min(max(w[0], 0.0), W - 1.0)
                y = min(max(w[1], 0.0), H - 1.0)
                out[v, u] = bilinear(I_t, np.array([x]), np.array([y]))[0]
    return out
