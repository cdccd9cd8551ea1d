"""ctypes wrapper of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark. The product path never imports it.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

KEYFRAME_DUE, DIVERGED, LOW_OVERLAP = 1, 2, 4


class OrConfig(C.Structure):
    _fields_ = [
        ("H", C.c_int), ("W", C.c_int),
        ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
        ("sigma_D", C.c_double), ("sigma_P", C.c_double), ("sigma_R", C.c_double),
        ("sigma_N", C.c_double), ("huber_k", C.c_double),
        ("init_inv_depth", C.c_double),
        ("prior_xi", C.c_double * 6), ("prior_log_depth", C.c_double),
        ("kf_max_frames", C.c_int), ("kf_min_valid_frac", C.c_double),
        ("damping", C.c_double),
        ("frozen", C.c_int), ("full_jacobian", C.c_int),
        ("topology", C.c_int),
        ("store_fp32", C.c_int),
    ]


TOPO_GRID, TOPO_QUADTREE = 0, 1


class OrTrackOut(C.Structure):
    _fields_ = [
        ("xi", C.c_double * 6), ("T_world", C.c_double * 16),
        ("valid_fraction", C.c_double), ("frames_since_keyframe", C.c_int),
        ("flags", C.c_uint),
    ]


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = load(LIB_PATH)
    return _lib


def load(path: str) -> C.CDLL:
    """Loads an oracle library built from pixvod_oracle.c (the oracle itself, or
    a variant the tests build with a planted fault) and declares its calls."""
    L = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    fp = C.POINTER(C.c_float)
    L.or_create.restype = C.c_void_p
    L.or_create.argtypes = [C.POINTER(OrConfig)]
    L.or_destroy.argtypes = [C.c_void_p]
    L.or_default_config.argtypes = [C.POINTER(OrConfig)]
    L.or_set_sigma_D_map.argtypes = [C.c_void_p, dp]
    L.or_set_prior.argtypes = [C.c_void_p, dp, dp]
    L.or_set_prior_from_state.argtypes = [C.c_void_p]
    L.or_set_keyframe.argtypes = [C.c_void_p, fp, fp]
    L.or_track.argtypes = [C.c_void_p, fp, C.c_int, C.POINTER(OrTrackOut), dp, dp]
    L.or_iterate.argtypes = [C.c_void_p, C.c_int]
    L.or_set_keyframe64.argtypes = [C.c_void_p, dp, fp]
    L.or_set_frame64.argtypes = [C.c_void_p, dp]
    L.or_set_frame.argtypes = [C.c_void_p, fp]
    L.or_state_doubles.restype = C.c_size_t
    L.or_state_doubles.argtypes = [C.c_void_p]
    L.or_get_state.argtypes = [C.c_void_p, dp]
    L.or_set_state.argtypes = [C.c_void_p, dp]
    L.or_get_means.argtypes = [C.c_void_p, dp]
    L.or_get_beliefs.argtypes = [C.c_void_p, dp, dp]
    L.or_get_normal_targets.argtypes = [C.c_void_p, dp, dp]
    L.or_get_gradients.argtypes = [C.c_void_p, dp, dp]
    L.or_transfer_depth.argtypes = [C.c_void_p]
    L.or_tree_levels.restype = C.c_int
    L.or_tree_levels.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
    L.or_get_node_beliefs.argtypes = [C.c_void_p, dp, dp]
    L.or_energy.restype = C.c_double
    L.or_energy.argtypes = [C.c_void_p]
    L.or_se3_exp.argtypes = [dp, dp]
    L.or_se3_log.argtypes = [dp, dp]
    L.or_se3_jr.argtypes = [dp, dp]
    L.or_prior_jacobian.argtypes = [dp, dp]
    L.or_huber_weight.restype = C.c_double
    L.or_huber_weight.argtypes = [C.c_double, C.c_double]
    L.or_warp.argtypes = [C.c_void_p, C.c_double, C.c_double, dp, C.c_double, dp, dp]
    L.or_unary.argtypes = [C.c_void_p, C.c_int, C.c_int, dp, dp, C.POINTER(C.c_int)]
    L.or_factor_message.argtypes = [C.c_int, dp, dp, dp, dp, dp, dp, dp]
    L.or_threads.restype = C.c_int
    L.or_set_threads.argtypes = [C.c_int]
    return L


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _fp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def default_config(**kw) -> OrConfig:
    cfg = OrConfig()
    lib().or_default_config(C.byref(cfg))
    for k, v in kw.items():
        if k == "prior_xi":
            for i in range(6):
                cfg.prior_xi[i] = float(v[i])
        else:
            setattr(cfg, k, v)
    return cfg


def config_for_camera(cam, **kw) -> OrConfig:
    return default_config(H=cam.H, W=cam.W, fx=cam.fx, fy=cam.fy, cx=cam.cx, cy=cam.cy, **kw)


# ---------------------------------------------------------------------------
# building blocks


def se3_exp(xi) -> np.ndarray:
    x = np.ascontiguousarray(xi, dtype=np.float64)
    T = np.zeros(16)
    lib().or_se3_exp(_dp(x), _dp(T))
    return T.reshape(4, 4)


def se3_log(T) -> np.ndarray:
    t = np.ascontiguousarray(np.asarray(T, dtype=np.float64).reshape(16))
    xi = np.zeros(6)
    lib().or_se3_log(_dp(t), _dp(xi))
    return xi


def se3_jr(xi) -> np.ndarray:
    x = np.ascontiguousarray(xi, dtype=np.float64)
    J = np.zeros(36)
    lib().or_se3_jr(_dp(x), _dp(J))
    return J.reshape(6, 6)


def prior_jacobian(xi) -> np.ndarray:
    x = np.ascontiguousarray(xi, dtype=np.float64)
    J = np.zeros(36)
    lib().or_prior_jacobian(_dp(x), _dp(J))
    return J.reshape(6, 6)


def huber_weight(M: float, k: float) -> float:
    return lib().or_huber_weight(float(M), float(k))


def factor_message(r, J, prec, eta_s, lam_s):
    r = np.ascontiguousarray(np.atleast_1d(r), dtype=np.float64)
    m = r.shape[0]
    J = np.ascontiguousarray(np.asarray(J, dtype=np.float64).reshape(m, 14))
    prec = np.ascontiguousarray(np.atleast_1d(prec), dtype=np.float64)
    eta_s = np.ascontiguousarray(eta_s, dtype=np.float64)
    lam_s = np.ascontiguousarray(np.asarray(lam_s, dtype=np.float64).reshape(49))
    eo, lo = np.zeros(7), np.zeros(49)
    rc = lib().or_factor_message(m, _dp(r), _dp(J), _dp(prec), _dp(eta_s), _dp(lam_s), _dp(eo), _dp(lo))
    if rc != 0:
        raise ValueError("singular sender block")
    return eo, lo.reshape(7, 7)


# ---------------------------------------------------------------------------
# the iteration


class Oracle:
    """One oracle context: keyframe, target frames, GBP state (FP64)."""

    def __init__(self, cfg: OrConfig, library: Optional[C.CDLL] = None):
        self.cfg = cfg
        self.H, self.W = cfg.H, cfg.W
        self._L = library if library is not None else lib()
        self._h = self._L.or_create(C.byref(cfg))
        if not self._h:
            raise ValueError("invalid oracle configuration")

    def close(self):
        if self._h:
            self._L.or_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def N(self) -> int:
        return self.H * self.W

    def set_sigma_D_map(self, sig: Optional[np.ndarray]):
        if sig is None:
            self._L.or_set_sigma_D_map(self._h, None)
        else:
            s = np.ascontiguousarray(sig, dtype=np.float64).reshape(self.N)
            self._L.or_set_sigma_D_map(self._h, _dp(s))

    def set_prior(self, xi=None, log_depth=None):
        """Prior means: pose xi (6) and per-pixel log-depths (H x W); None keeps them."""
        x = None if xi is None else np.ascontiguousarray(xi, dtype=np.float64)
        d = None if log_depth is None else np.ascontiguousarray(log_depth, dtype=np.float64).reshape(self.N)
        self._L.or_set_prior(self._h, None if x is None else _dp(x), None if d is None else _dp(d))

    def set_prior_from_state(self):
        """Temporal priors: the current mean pose and log-depths become the prior means."""
        self._L.or_set_prior_from_state(self._h)

    def set_keyframe(self, img, normals):
        i = np.ascontiguousarray(img, dtype=np.float32).reshape(self.N)
        n = np.ascontiguousarray(normals, dtype=np.float32).reshape(self.N * 3)
        rc = self._L.or_set_keyframe(self._h, _fp(i), _fp(n))
        assert rc == 0

    def transfer_depth(self):
        """Forward-warps the log-depths into the frame just tracked (call
        before set_keyframe with that frame)."""
        rc = self._L.or_transfer_depth(self._h)
        if rc != 0:
            raise RuntimeError("depth transfer needs a tracked frame")

    def set_keyframe64(self, img, normals):
        i = np.ascontiguousarray(img, dtype=np.float64).reshape(self.N)
        n = np.ascontiguousarray(normals, dtype=np.float32).reshape(self.N * 3)
        assert self._L.or_set_keyframe64(self._h, _dp(i), _fp(n)) == 0

    def set_frame64(self, frame):
        f = np.ascontiguousarray(frame, dtype=np.float64).reshape(self.N)
        self._L.or_set_frame64(self._h, _dp(f))

    def set_frame(self, frame):
        f = np.ascontiguousarray(frame, dtype=np.float32).reshape(self.N)
        self._L.or_set_frame(self._h, _fp(f))

    def iterate(self, n: int) -> int:
        return self._L.or_iterate(self._h, int(n))

    def track(self, frame, n_iters: int):
        f = np.ascontiguousarray(frame, dtype=np.float32).reshape(self.N)
        out = OrTrackOut()
        inv = np.zeros(self.N)
        var = np.zeros(self.N)
        rc = self._L.or_track(self._h, _fp(f), int(n_iters), C.byref(out), _dp(inv), _dp(var))
        if rc != 0:
            raise RuntimeError(f"or_track failed: {rc}")
        return dict(xi=np.array(out.xi[:]), T_world=np.array(out.T_world[:]).reshape(4, 4),
                    valid_fraction=out.valid_fraction,
                    frames_since_keyframe=out.frames_since_keyframe, flags=out.flags,
                    inv_depth=inv.reshape(self.H, self.W), inv_depth_var=var.reshape(self.H, self.W))

    @property
    def tree(self) -> bool:
        return self.cfg.topology == TOPO_QUADTREE

    def tree_levels(self):
        """[(rows, cols)] of levels 0 (pixels) .. L (root); [(H, W)] for the grid."""
        hw = (C.c_int * 64)()
        L = self._L.or_tree_levels(self._h, hw)
        return [(hw[2 * l], hw[2 * l + 1]) for l in range(L + 1)]

    @property
    def n_nodes(self) -> int:
        return sum(h * w for h, w in self.tree_levels()[1:])

    def get_state(self):
        """Grid: (H, W, 123). Quadtree: ((H, W, 42) pixel part, (n_nodes, 141) node part)."""
        n = self._L.or_state_doubles(self._h)
        s = np.zeros(n)
        self._L.or_get_state(self._h, _dp(s))
        if not self.tree:
            return s.reshape(self.H, self.W, 123)
        return s[:self.N * 42].reshape(self.H, self.W, 42), s[self.N * 42:].reshape(-1, 141)

    def set_state(self, s):
        if self.tree:
            pix, nodes = s
            s = np.concatenate([np.asarray(pix, dtype=np.float64).reshape(-1),
                                np.asarray(nodes, dtype=np.float64).reshape(-1)])
        s = np.ascontiguousarray(s, dtype=np.float64).reshape(-1)
        assert s.size == self._L.or_state_doubles(self._h)
        self._L.or_set_state(self._h, _dp(s))

    def node_beliefs(self):
        n = self.n_nodes
        lam = np.zeros(n * 49)
        eta = np.zeros(n * 7)
        self._L.or_get_node_beliefs(self._h, _dp(lam), _dp(eta))
        return lam.reshape(n, 7, 7), eta.reshape(n, 7)

    def means(self) -> np.ndarray:
        m = np.zeros(self.N * 7)
        self._L.or_get_means(self._h, _dp(m))
        return m.reshape(self.H, self.W, 7)

    def beliefs(self):
        lam = np.zeros(self.N * 49)
        eta = np.zeros(self.N * 7)
        self._L.or_get_beliefs(self._h, _dp(lam), _dp(eta))
        return lam.reshape(self.H, self.W, 7, 7), eta.reshape(self.H, self.W, 7)

    def normal_targets(self):
        cx, cy = np.zeros(self.N), np.zeros(self.N)
        self._L.or_get_normal_targets(self._h, _dp(cx), _dp(cy))
        return cx.reshape(self.H, self.W), cy.reshape(self.H, self.W)

    def gradients(self):
        gx, gy = np.zeros(self.N), np.zeros(self.N)
        self._L.or_get_gradients(self._h, _dp(gx), _dp(gy))
        return gx.reshape(self.H, self.W), gy.reshape(self.H, self.W)

    def energy(self) -> float:
        return self._L.or_energy(self._h)

    def warp(self, u: float, v: float, tau, ell: float):
        t = np.ascontiguousarray(tau, dtype=np.float64)
        w, J = np.zeros(2), np.zeros(14)
        ok = self._L.or_warp(self._h, float(u), float(v), _dp(t), float(ell), _dp(w), _dp(J))
        return bool(ok), w, J.reshape(2, 7)

    def unary(self, u: int, v: int):
        eta, lam = np.zeros(7), np.zeros(49)
        valid = C.c_int(0)
        rc = self._L.or_unary(self._h, int(u), int(v), _dp(eta), _dp(lam), C.byref(valid))
        assert rc == 0
        return eta, lam.reshape(7, 7), bool(valid.value)


def threads() -> int:
    return lib().or_threads()


def set_threads(n: int):
    """Threads of the oracle's OpenMP loops from now on."""
    lib().or_set_threads(int(n))
