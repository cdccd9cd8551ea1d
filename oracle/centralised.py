"""Centralised direct tracking by IRLS Gauss-Newton (Sec. 3.1, Eq. photo, and
the centralised baseline of Sec. 4.4, Fig. centralized_vs_pixvod).

TEST INFRASTRUCTURE ONLY: the reference that the GPU's centralised solver is
checked against. It shares no code with the GPU library.

One global relative pose xi (se(3), right perturbation T = Exp(xi) Exp(d))
and a log-depth per keyframe pixel, with every measurement accessible at
once. The energy is Eq. (photo) with the per-pixel model's factors at exact
consensus: every pixel's pose equals xi, so there are no identity factors;
each pixel keeps its photometric factor (Eq. distrb_photo, Huber by
iteratively reweighted least squares: the weight kappa of the Huber
covariance weighting at the current residual), its log-depth prior and the
normal-integration factors (Eq. gbpni); the one pose has one prior factor
(Eq. prior) of the same strength. One IRLS iteration
solves the Gauss-Newton normal equations of the model linearised at the
current point, with the weights frozen there, exactly (sparse direct solve),
and applies the step: xi <- Log(Exp(xi) Exp(d_xi)), ell <- ell + d_ell.

Unknowns are ordered [d_xi (6); d_ell (N)], pixels row-major.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .dense import WARP_EPS, bilinear, exp_se3, gradients, huber_kappa, log_se3, normal_targets, prior_jac


class Centralised:
    def __init__(self, H, W, K, I_s, normals, sigma_D=5e-3, sigma_P=1.0, sigma_N=1e-3, huber_k=400.0,
                 prior_xi=None, prior_log_depth=0.0, sigma_D_map=None):
        self.H, self.W = H, W
        self.K = tuple(float(k) for k in K)
        self.I_s = np.asarray(I_s, np.float64).reshape(H, W)
        self.cxt, self.cyt = normal_targets(np.asarray(normals, np.float32).reshape(H, W, 3), self.K)
        self.sigD = np.full((H, W), float(sigma_D)) if sigma_D_map is None else np.asarray(sigma_D_map, np.float64)
        self.lamP = float(sigma_P) ** -2
        self.lamN = 0.0 if math.isinf(sigma_N) else float(sigma_N) ** -2
        self.k = float(huber_k)
        self.prior_xi = np.zeros(6) if prior_xi is None else np.asarray(prior_xi, np.float64)
        self.prior_ell = np.broadcast_to(np.asarray(prior_log_depth, np.float64), (H, W)).reshape(-1).copy()
        self.I_t = None

    @property
    def N(self):
        return self.H * self.W

    def set_frame(self, I_t):
        self.I_t = np.asarray(I_t, np.float64).reshape(self.H, self.W)
        self.Gx, self.Gy = gradients(self.I_t)

    # -- the photometric factor of every pixel at the shared pose ---------------
    def photometric(self, xi, ell):
        """valid (N,), residual r (N,), Jacobian rows J (N, 7) with respect to
        [d_xi; d_ell_i], IRLS weight kappa * Lambda_D (N,)."""
        fx, fy, cx, cy = self.K
        H, W = self.H, self.W
        T = exp_se3(xi)
        R, t = T[:3, :3], T[:3, 3]
        u, v = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
        q = np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u)], -1).reshape(-1, 3)
        rho = np.exp(-np.asarray(ell, np.float64).reshape(-1))
        a = q @ R.T + rho[:, None] * t[None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            wx = fx * a[:, 0] / a[:, 2] + cx
            wy = fy * a[:, 1] / a[:, 2] + cy
        valid = (a[:, 2] > 0) & (wx >= -WARP_EPS) & (wx <= W - 1 + WARP_EPS) & (wy >= -WARP_EPS) & \
            (wy <= H - 1 + WARP_EPS)
        x = np.clip(np.where(valid, wx, 0.0), 0.0, W - 1.0)
        y = np.clip(np.where(valid, wy, 0.0), 0.0, H - 1.0)
        It = bilinear(self.I_t, x, y)
        gx = bilinear(self.Gx, x, y)
        gy = bilinear(self.Gy, x, y)
        r = self.I_s.reshape(-1) - It
        az = np.where(valid, a[:, 2], 1.0)
        # dw/da (2 x 3 per pixel) and da/d[d_theta, d_rho, d_ell] = [-R [q]x, rho R, -rho t]
        d0 = np.stack([fx / az, np.zeros_like(az), -fx * a[:, 0] / az ** 2], -1)
        d1 = np.stack([np.zeros_like(az), fy / az, -fy * a[:, 1] / az ** 2], -1)
        c = -(gx[:, None] * d0 + gy[:, None] * d1)              # -g^T dw/da, (N, 3)
        J = np.zeros((self.N, 7))
        Rt_c = c @ R                                            # R^T c per pixel
        # c . (-R [q]x d) = -(R^T c) . (q x d) = -((R^T c) x q) . d  ... as a row: (q x R^T c)
        J[:, :3] = np.cross(q, Rt_c)
        J[:, 3:6] = rho[:, None] * Rt_c
        J[:, 6] = -rho * (c @ t)
        lamD = self.sigD.reshape(-1) ** -2
        kap = huber_kappa(np.abs(r) * np.sqrt(lamD), self.k)
        wgt = np.where(valid, kap * lamD, 0.0)
        return valid, np.where(valid, r, 0.0), J, wgt

    def normal_edges(self):
        """(a, b, c) of every active normal-integration edge, a the left/upper pixel."""
        H, W = self.H, self.W
        idx = np.arange(self.N).reshape(H, W)
        a_h, b_h, c_h = idx[:, :-1].reshape(-1), idx[:, 1:].reshape(-1), self.cxt[:, :-1].reshape(-1)
        a_v, b_v, c_v = idx[:-1, :].reshape(-1), idx[1:, :].reshape(-1), self.cyt[:-1, :].reshape(-1)
        a = np.concatenate([a_h, a_v])
        b = np.concatenate([b_h, b_v])
        c = np.concatenate([c_h, c_v])
        ok = np.isfinite(c)
        return a[ok], b[ok], c[ok]

    def normal_equations(self, xi, ell):
        """Sparse (N + 6) x (N + 6) Gauss-Newton matrix M and right-hand side g
        (M d = g, g = -J^T Lambda r) at (xi, ell); also the valid count."""
        N = self.N
        ell = np.asarray(ell, np.float64).reshape(-1)
        valid, r, J, w = self.photometric(xi, ell)
        Jx, Jl = J[:, :6], J[:, 6]
        A = (Jx * w[:, None]).T @ Jx
        gx = -(Jx * (w * r)[:, None]).sum(0)
        # the prior factor of the one pose
        rp = log_se3(np.linalg.inv(exp_se3(self.prior_xi)) @ exp_se3(xi))
        Jp = prior_jac(rp)
        A = A + self.lamP * Jp.T @ Jp
        A = 0.5 * (A + A.T)          # symmetric by definition; drop the rounding asymmetry
        gx = gx - self.lamP * Jp.T @ rp
        Bc = Jx * (w * Jl)[:, None]                             # (N, 6) coupling
        dg = w * Jl * Jl + self.lamP
        gl = -w * Jl * r - self.lamP * (ell - self.prior_ell)
        a, b, c = self.normal_edges()
        lam = self.lamN
        rows, cols, vals = [], [], []
        if lam > 0 and a.size:
            rn = ell[b] - ell[a] + c
            np.add.at(dg, a, lam)
            np.add.at(dg, b, lam)
            np.add.at(gl, b, -lam * rn)
            np.add.at(gl, a, lam * rn)
            rows += [6 + a, 6 + b]
            cols += [6 + b, 6 + a]
            vals += [np.full(a.size, -lam), np.full(a.size, -lam)]
        pix = 6 + np.arange(N)
        rows += [pix]
        cols += [pix]
        vals += [dg]
        for k in range(6):
            rows += [np.full(N, k), pix]
            cols += [pix, np.full(N, k)]
            vals += [Bc[:, k], Bc[:, k]]
        ii, jj = np.meshgrid(np.arange(6), np.arange(6), indexing="ij")
        rows += [ii.reshape(-1)]
        cols += [jj.reshape(-1)]
        vals += [A.reshape(-1)]
        M = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N + 6, N + 6))
        g = np.concatenate([gx, gl])
        return M, g, int(valid.sum())

    def step(self, xi, ell):
        """The exact Gauss-Newton step (d_xi (6), d_ell (N)) at (xi, ell), by
        block elimination of the depths: with M = [[A, B], [B', D]] and one
        sparse LU factorisation of D, S = A - B D^-1 B', d_xi = S^-1 (g_xi -
        B D^-1 g_ell), d_ell = D^-1 (g_ell - B' d_xi)."""
        M, g, _ = self.normal_equations(xi, ell)
        M = M.tocsc()
        A = M[:6, :6].toarray()
        B = M[:6, 6:].toarray()
        lu = spla.splu(M[6:, 6:].tocsc())
        Y = lu.solve(np.ascontiguousarray(B.T))
        y = lu.solve(g[6:])
        S = A - B @ Y
        dx = np.linalg.solve(S, g[:6] - B @ y)
        return dx, y - Y @ dx

    def iterate(self, xi, ell, n_iters: int):
        xi = np.array(xi, np.float64)
        ell = np.array(ell, np.float64).reshape(-1)
        for _ in range(n_iters):
            dx, dl = self.step(xi, ell)
            xi = log_se3(exp_se3(xi) @ exp_se3(dx))
            ell = ell + dl
        return xi, ell
