"""Gradients of unrolled oracle tracking by central finite differences (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): the reference the GPU
adjoint is checked against. An unrolled run starts from a fresh keyframe
state, tracks F target frames with a fixed iteration count each (no
re-anchoring) and reports per frame the pose estimate xi (mean of the
per-pixel pose tangents, Eq. estimator_avg) and the inverse-depth map. For
output cotangents (cxi, crho) the scalar
    L = sum_f cxi[f] . xi[f] + sum_f sum_i crho[f, i] rho[f, i]
is differentiated with respect to the photometric sigma map (Eq.
distrb_photo), the normal-integration sigma (Eq. gbpni) and the Huber
threshold by symmetric differences of relative step h. A run may start from
a given state instead of the fresh keyframe state (teacher forcing: a few
iterations from the same state on both sides of a comparison).
"""

from __future__ import annotations

from typing import Dict, Optional

import numpy as np

from . import Oracle, config_for_camera


class UnrolledOracle:
    """Repeated unrolled runs of one workload with varying parameters."""

    def __init__(self, cam, I_s, N_s, frames, n_iters: int, sigma_map, sigma_N: float, huber_k: float,
                 start=None, **cfg_kw):
        self.cam, self.I_s, self.N_s = cam, I_s, N_s
        self.start = None if start is None else np.asarray(start, np.float64)
        self.frames = [np.asarray(f, np.float32) for f in frames]
        self.n_iters = int(n_iters)
        self.sigma_map = np.asarray(sigma_map, np.float64)
        self.sigma_N, self.huber_k = float(sigma_N), float(huber_k)
        self.cfg_kw = cfg_kw

    def outputs(self, sigma_map=None, sigma_N=None, huber_k=None) -> Dict[str, np.ndarray]:
        cfg = config_for_camera(self.cam, sigma_N=self.sigma_N if sigma_N is None else sigma_N,
                                huber_k=self.huber_k if huber_k is None else huber_k, **self.cfg_kw)
        o = Oracle(cfg)
        try:
            o.set_sigma_D_map(self.sigma_map if sigma_map is None else sigma_map)
            o.set_keyframe(self.I_s, self.N_s)
            if self.start is not None:
                o.set_state(self.start)
            xi, rho = [], []
            for f in self.frames:
                r = o.track(f, self.n_iters)
                xi.append(r["xi"])
                rho.append(r["inv_depth"])
        finally:
            o.close()
        return dict(xi=np.array(xi), inv_depth=np.array(rho))

    @staticmethod
    def functional(out, cxi, crho) -> float:
        return float(np.sum(np.asarray(cxi) * out["xi"]) + np.sum(np.asarray(crho, np.float64) * out["inv_depth"]))

    def loss(self, cxi, crho, **kw) -> float:
        return self.functional(self.outputs(**kw), cxi, crho)

    def d_sigma_N(self, cxi, crho, h: float = 1e-6) -> float:
        s = self.sigma_N
        return (self.loss(cxi, crho, sigma_N=s * (1 + h)) - self.loss(cxi, crho, sigma_N=s * (1 - h))) / (2 * h * s)

    def d_huber_k(self, cxi, crho, h: float = 1e-6) -> float:
        k = self.huber_k
        return (self.loss(cxi, crho, huber_k=k * (1 + h)) - self.loss(cxi, crho, huber_k=k * (1 - h))) / (2 * h * k)

    def d_sigma_entry(self, cxi, crho, v: int, u: int, h: float = 1e-6) -> float:
        s = self.sigma_map[v, u]
        mp = self.sigma_map.copy()
        mm = self.sigma_map.copy()
        mp[v, u] = s * (1 + h)
        mm[v, u] = s * (1 - h)
        return (self.loss(cxi, crho, sigma_map=mp) - self.loss(cxi, crho, sigma_map=mm)) / (2 * h * s)

    def d_direction(self, cxi, crho, d_map: np.ndarray, d_N: float, d_k: float, h: float = 1e-6) -> float:
        """Directional derivative along relative changes: sigma_map * (1 + t d_map),
        sigma_N (1 + t d_N), huber_k (1 + t d_k) at t = 0."""
        def at(t):
            return self.loss(cxi, crho, sigma_map=self.sigma_map * (1 + t * d_map),
                             sigma_N=self.sigma_N * (1 + t * d_N), huber_k=self.huber_k * (1 + t * d_k))
        return (at(h) - at(-h)) / (2 * h)


def central_difference(f, x: float, h: float) -> float:
    """Symmetric difference quotient of a scalar function (absolute step h)."""
    return (f(x + h) - f(x - h)) / (2 * h)


def relative_sensitivity(f, x: float, hs=(1e-5, 1e-6)) -> Optional[float]:
    """Spread of relative-step difference quotients over the steps hs, relative
    to the last one: a smoothness indicator of f around x."""
    g = [(f(x * (1 + h)) - f(x * (1 - h))) / (2 * h * x) for h in hs]
    return float(np.ptp(g) / max(abs(g[-1]), 1e-300))
