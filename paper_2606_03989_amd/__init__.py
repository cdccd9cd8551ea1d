"""Python binding of libpixvod: per-pixel GBP visual odometry and depth on MI355X.

Argument marshalling only: every step of the method runs in the HIP kernels of
libpixvod.so. torch is imported before the library is loaded so that torch
and libpixvod share one HIP runtime; torch tensors on the GPU are passed as
device pointers on the context's stream, numpy arrays and CPU tensors as host
pointers.

The library must be built (``python -m paper_2606_03989_amd.build`` or
``__graft_entry__.build()``); importing this package without it raises.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np
import torch  # noqa: F401  (shared HIP runtime; must precede the library load)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpixvod.so")

OK, EINVAL, ESTATE, EHIP, ENOMEM, ENODEV = 0, -1, -2, -3, -4, -5
HOST, DEVICE = 0, 1
KEYFRAME_DUE, DIVERGED, LOW_OVERLAP = 1, 2, 4
SCHED_FUSED, SCHED_PER_FACTOR = 0, 1
PROF_FUSED_ITERATE, PROF_FUSED_FINAL, PROF_FUSED_PROLOGUE, PROF_PER_FACTOR = 0, 1, 2, 3
N_PLANES = 123
TOPO_GRID, TOPO_QUADTREE = 0, 1
TREE_PIXEL_PLANES, TREE_NODE_PLANES = 42, 141


class PixvodError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pixvod error {code}: {msg}")
        self.code = code


class Intrinsics(C.Structure):
    _fields_ = [("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float)]


class Params(C.Structure):
    _fields_ = [
        ("sigma_D", C.c_float), ("sigma_P", C.c_float), ("sigma_R", C.c_float), ("sigma_N", C.c_float),
        ("huber_k", C.c_float), ("init_inv_depth", C.c_float), ("prior_xi", C.c_float * 6),
        ("prior_log_depth", C.c_float), ("kf_max_frames", C.c_int32), ("kf_min_valid_frac", C.c_float),
        ("damping", C.c_float),
    ]


class TrackOut(C.Structure):
    _fields_ = [
        ("xi_rel", C.c_double * 6), ("T_world", C.c_double * 16),
        ("inv_depth", C.c_void_p), ("inv_depth_var", C.c_void_p), ("out_where", C.c_int32),
        ("valid_fraction", C.c_float), ("frames_since_keyframe", C.c_int32), ("flags", C.c_uint32),
    ]


class CentralStats(C.Structure):
    _fields_ = [("cg_iters", C.c_int32), ("last_cg_iters", C.c_int32), ("last_rel_residual", C.c_double),
                ("valid_fraction", C.c_float), ("flags", C.c_uint32)]


_lib: Optional[C.CDLL] = None

# every entry point declared in include/pixvod.h, with its ctypes signature
_SIGNATURES = {
    "pixvod_default_params": (None, [C.POINTER(Params)]),
    "pixvod_create": (C.c_int, [C.c_int, C.c_int, C.POINTER(Intrinsics), C.POINTER(Params), C.POINTER(C.c_void_p)]),
    "pixvod_destroy": (C.c_int, [C.c_void_p]),
    "pixvod_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pixvod_set_schedule": (C.c_int, [C.c_void_p, C.c_int]),
    "pixvod_set_topology": (C.c_int, [C.c_void_p, C.c_int]),
    "pixvod_tree_levels": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "pixvod_set_keyframe": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "pixvod_set_sigma_map": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "pixvod_set_keyframe_transfer": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "pixvod_set_keyframe_transfer_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "pixvod_track": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.POINTER(TrackOut)]),
    "pixvod_iterate": (C.c_int, [C.c_void_p, C.c_int]),
    "pixvod_set_prior": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "pixvod_set_prior_from_state": (C.c_int, [C.c_void_p]),
    "pixvod_state_bytes": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "pixvod_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "pixvod_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "pixvod_profile_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "pixvod_set_graph": (C.c_int, [C.c_void_p, C.c_int]),
    "pixvod_profile_read": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "pixvod_batch_create": (C.c_int, [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(Intrinsics),
                                      C.POINTER(Params), C.POINTER(C.c_void_p)]),
    "pixvod_batch_destroy": (C.c_int, [C.c_void_p]),
    "pixvod_batch_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pixvod_batch_set_keyframes": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_void_p),
                                             C.POINTER(C.c_void_p), C.c_int]),
    "pixvod_batch_track": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.c_int, C.c_int, C.POINTER(TrackOut)]),
    "pixvod_batch_track_reanchor": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int,
                                              C.c_int, C.POINTER(TrackOut)]),
    "pixvod_batch_set_persistent": (C.c_int, [C.c_void_p, C.c_int]),
    "pixvod_batch_set_tile": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "pixvod_batch_autotune": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "pixvod_batch_last_step_ms": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "pixvod_batch_get_state": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int]),
    "pixvod_batch_set_state": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int]),
    "pixvod_unroll_create": (C.c_int, [C.c_int, C.c_int, C.POINTER(Intrinsics), C.POINTER(Params), C.c_int, C.c_int,
                                       C.c_int, C.POINTER(C.c_void_p)]),
    "pixvod_unroll_destroy": (C.c_int, [C.c_void_p]),
    "pixvod_unroll_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pixvod_unroll_set_keyframe": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "pixvod_unroll_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "pixvod_unroll_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_double,
                                        C.c_double, C.c_void_p, C.c_void_p, C.c_int]),
    "pixvod_unroll_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                                         C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pixvod_unroll_last_ms": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pixvod_central_create": (C.c_int, [C.c_int, C.c_int, C.POINTER(Intrinsics), C.POINTER(Params), C.c_int,
                                        C.c_double, C.POINTER(C.c_void_p)]),
    "pixvod_central_destroy": (C.c_int, [C.c_void_p]),
    "pixvod_central_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pixvod_central_set_keyframe": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "pixvod_central_set_point": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pixvod_central_get_point": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pixvod_central_track": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                                       C.POINTER(CentralStats)]),
    "pixvod_central_last_ms": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "pixvod_last_error": (C.c_char_p, [C.c_void_p]),
    "pixvod_version": (C.c_char_p, []),
}


def lib() -> C.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libpixvod.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def default_params(**overrides) -> Params:
    p = Params()
    lib().pixvod_default_params(C.byref(p))
    for k, v in overrides.items():
        if k == "prior_xi":
            for i in range(6):
                p.prior_xi[i] = float(v[i])
        else:
            setattr(p, k, v)
    return p


def _check(rc: int, ctx=None):
    if rc != OK:
        msg = lib().pixvod_last_error(ctx)
        raise PixvodError(rc, msg.decode() if msg else "")


def _ptr(a, dtype=np.float32):
    """(pointer, where, keepalive) for a numpy array or torch tensor."""
    if isinstance(a, torch.Tensor):
        if a.dtype != torch.float32:
            raise TypeError("float32 tensors required")
        if not a.is_contiguous():
            raise ValueError("contiguous tensors required")
        return a.data_ptr(), (DEVICE if a.is_cuda else HOST), a
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data, HOST, arr


class _FollowsTorchStream:
    """Stream binding shared by the wrappers. A call that takes or returns
    CUDA tensors runs on torch's current stream, so it is ordered after the
    torch work that produced its inputs and before the work that reads its
    outputs, unless set_stream() chose a stream explicitly. Binding a new
    stream waits for the work already queued on the previous one."""

    _explicit_stream = False
    _bound_stream = None

    def _bind_stream(self, handle):
        raise NotImplementedError

    def set_stream(self, stream=None):
        s = None if stream is None else (stream.cuda_stream if hasattr(stream, "cuda_stream") else stream)
        self._bind_stream(None if s is None else C.c_void_p(s))
        self._explicit_stream = s is not None
        self._bound_stream = s

    def _follow_torch(self, *wheres):
        if self._explicit_stream or DEVICE not in wheres:
            return
        cur = torch.cuda.current_stream().cuda_stream
        if cur != self._bound_stream:
            self._bind_stream(C.c_void_p(cur))
            self._bound_stream = cur


class Tracker(_FollowsTorchStream):
    """One image sequence: keyframe, target frames and the GBP state on the GPU."""

    def __init__(self, H: int, W: int, K, params: Optional[Params] = None, **overrides):
        self.H, self.W = int(H), int(W)
        if params is None:
            params = default_params(**overrides)
        self.params = params
        Kc = Intrinsics(*[float(x) for x in K])
        h = C.c_void_p()
        _check(lib().pixvod_create(self.H, self.W, C.byref(Kc), C.byref(params), C.byref(h)))
        self._h = h
        self.topology = TOPO_GRID

    def close(self):
        if getattr(self, "_h", None):
            lib().pixvod_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _bind_stream(self, handle):
        _check(lib().pixvod_set_stream(self._h, handle), self._h)

    def set_schedule(self, schedule: int):
        _check(lib().pixvod_set_schedule(self._h, int(schedule)), self._h)

    def set_keyframe(self, img, normals, transfer_depth: bool = False, noalloc: bool = False):
        """New keyframe; with transfer_depth the log-depths are first
        forward-warped into it (img should be the frame just tracked);
        noalloc selects the transfer's allocation-free entry point."""
        pi, wi, ki = _ptr(img)
        pn, wn, kn = _ptr(normals)
        if wi != wn:
            raise ValueError("image and normals must live in the same memory")
        if noalloc and not transfer_depth:
            raise ValueError("noalloc applies to the depth-transfer re-anchoring")
        if transfer_depth:
            f = lib().pixvod_set_keyframe_transfer_noalloc if noalloc else lib().pixvod_set_keyframe_transfer
        else:
            f = lib().pixvod_set_keyframe
        self._follow_torch(wi)
        _check(f(self._h, C.c_void_p(pi), C.c_void_p(pn), wi), self._h)

    def set_sigma_map(self, sigma):
        if sigma is None:
            _check(lib().pixvod_set_sigma_map(self._h, None, HOST), self._h)
            return
        p, w, k = _ptr(sigma)
        self._follow_torch(w)
        _check(lib().pixvod_set_sigma_map(self._h, C.c_void_p(p), w), self._h)

    def set_prior(self, xi=None, log_depth=None):
        """Prior means: pose xi (6) and per-pixel log-depths (H x W); None keeps them."""
        x = None if xi is None else np.ascontiguousarray(xi, dtype=np.float64)
        if log_depth is None:
            p, w, k = None, HOST, None
        else:
            p, w, k = _ptr(log_depth)
        self._follow_torch(w)
        _check(lib().pixvod_set_prior(self._h, None if x is None else C.c_void_p(x.ctypes.data),
                                      None if p is None else C.c_void_p(p), w), self._h)

    def set_prior_from_state(self):
        """Temporal priors: the last pose estimate and the current log-depths become the prior means."""
        _check(lib().pixvod_set_prior_from_state(self._h), self._h)

    def track(self, frame, n_iters: int, maps: bool = True, out_device: bool = False):
        """Tracks one frame; returns pose, world pose, flags and (optionally)
        the inverse-depth and variance maps (numpy, or torch CUDA tensors with
        out_device=True)."""
        pf, wf, kf = _ptr(frame)
        out = TrackOut()
        inv = var = None
        if maps:
            if out_device:
                inv = torch.empty((self.H, self.W), dtype=torch.float32, device="cuda")
                var = torch.empty((self.H, self.W), dtype=torch.float32, device="cuda")
                out.inv_depth, out.inv_depth_var, out.out_where = inv.data_ptr(), var.data_ptr(), DEVICE
            else:
                inv = np.empty((self.H, self.W), np.float32)
                var = np.empty((self.H, self.W), np.float32)
                out.inv_depth, out.inv_depth_var, out.out_where = inv.ctypes.data, var.ctypes.data, HOST
        else:
            out.out_where = HOST
        self._follow_torch(wf, out.out_where)
        _check(lib().pixvod_track(self._h, C.c_void_p(pf), wf, int(n_iters), C.byref(out)), self._h)
        return dict(xi=np.array(out.xi_rel[:]), T_world=np.array(out.T_world[:]).reshape(4, 4),
                    valid_fraction=float(out.valid_fraction),
                    frames_since_keyframe=int(out.frames_since_keyframe), flags=int(out.flags),
                    inv_depth=inv, inv_depth_var=var)

    def iterate(self, n: int):
        _check(lib().pixvod_iterate(self._h, int(n)), self._h)

    def profile(self, enable: bool = True):
        _check(lib().pixvod_profile_enable(self._h, 1 if enable else 0), self._h)

    def set_graph(self, enable: bool = True):
        """Replay the captured frame step, or launch every pass on its own (default)."""
        _check(lib().pixvod_set_graph(self._h, 1 if enable else 0), self._h)

    def profile_read(self, kind: int):
        """(total milliseconds, launches) of one timed pass kind; resets it."""
        ms, n = C.c_double(), C.c_int64()
        _check(lib().pixvod_profile_read(self._h, int(kind), C.byref(ms), C.byref(n)), self._h)
        return ms.value, n.value

    def state_bytes(self) -> int:
        n = C.c_size_t()
        _check(lib().pixvod_state_bytes(self._h, C.byref(n)), self._h)
        return n.value

    def set_topology(self, topology: int):
        """TOPO_GRID or TOPO_QUADTREE; before the first keyframe."""
        _check(lib().pixvod_set_topology(self._h, int(topology)), self._h)
        self.topology = int(topology)

    def tree_levels(self):
        """[(rows, cols)] of levels 0 (pixels) .. L (root); [(H, W)] for the grid."""
        n = C.c_int()
        hw = (C.c_int * 64)()
        _check(lib().pixvod_tree_levels(self._h, C.byref(n), hw), self._h)
        return [(hw[2 * l], hw[2 * l + 1]) for l in range(n.value)]

    def get_state(self):
        """Grid: (123, H, W) float32 (plane-major exchange layout). Quadtree:
        ((42, H, W) pixel planes, (141, NT) node planes)."""
        if self.topology == TOPO_QUADTREE:
            s = np.empty(self.state_bytes() // 4, np.float32)
            _check(lib().pixvod_get_state(self._h, C.c_void_p(s.ctypes.data), HOST), self._h)
            n = self.H * self.W * TREE_PIXEL_PLANES
            return s[:n].reshape(TREE_PIXEL_PLANES, self.H, self.W), s[n:].reshape(TREE_NODE_PLANES, -1)
        s = np.empty((N_PLANES, self.H, self.W), np.float32)
        _check(lib().pixvod_get_state(self._h, C.c_void_p(s.ctypes.data), HOST), self._h)
        return s

    def set_state(self, s):
        if isinstance(s, tuple):
            s = np.concatenate([np.asarray(s[0], np.float32).reshape(-1), np.asarray(s[1], np.float32).reshape(-1)])
            if s.size * 4 != self.state_bytes():
                raise ValueError("state size does not match the context")
        p, w, k = _ptr(s)
        self._follow_torch(w)
        _check(lib().pixvod_set_state(self._h, C.c_void_p(p), w), self._h)


def _batch_check(rc: int, h=None):
    if rc != OK:
        msg = lib().pixvod_last_error(None)
        raise PixvodError(rc, msg.decode() if msg else "")


class Batch(_FollowsTorchStream):
    """Many independent sequences (mixed resolutions) advanced together; one
    launch per pass over all sequences, frame steps replayed as HIP graphs."""

    def __init__(self, shapes, Ks, params: Optional[Params] = None, **overrides):
        self.shapes = [(int(h), int(w)) for h, w in shapes]
        n = len(self.shapes)
        if params is None:
            params = default_params(**overrides)
        self.params = params
        Hs = (C.c_int * n)(*[h for h, _ in self.shapes])
        Ws = (C.c_int * n)(*[w for _, w in self.shapes])
        Kc = (Intrinsics * n)(*[Intrinsics(*[float(x) for x in k]) for k in Ks])
        h = C.c_void_p()
        _batch_check(lib().pixvod_batch_create(n, Hs, Ws, Kc, C.byref(params), C.byref(h)))
        self._h = h
        self.n = n

    def close(self):
        if getattr(self, "_h", None):
            lib().pixvod_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind_stream(self, handle):
        _batch_check(lib().pixvod_batch_set_stream(self._h, handle))

    def set_keyframes(self, seq_ids, imgs, normals):
        m = len(seq_ids)
        keep, pi, pn, where = [], [], [], None
        for im, nm in zip(imgs, normals):
            a, wa, ka = _ptr(im)
            b, wb, kb = _ptr(nm)
            if where is None:
                where = wa
            if wa != where or wb != where:
                raise ValueError("all keyframe buffers must live in the same memory")
            keep += [ka, kb]
            pi.append(a)
            pn.append(b)
        ids = (C.c_int * m)(*seq_ids)
        self._follow_torch(where)
        _batch_check(lib().pixvod_batch_set_keyframes(self._h, m, ids, (C.c_void_p * m)(*pi), (C.c_void_p * m)(*pn),
                                                      HOST if where is None else where))

    def set_persistent(self, enable: bool = True):
        """Iteration block as one persistent cooperative launch (True) or one
        captured launch per pass (False, default)."""
        _batch_check(lib().pixvod_batch_set_persistent(self._h, 1 if enable else 0))

    def set_tile(self, tx: int, ty: int):
        _batch_check(lib().pixvod_batch_set_tile(self._h, int(tx), int(ty)))

    def autotune(self, n_iters: int):
        tx, ty = C.c_int(), C.c_int()
        _batch_check(lib().pixvod_batch_autotune(self._h, int(n_iters), C.byref(tx), C.byref(ty)))
        return tx.value, ty.value

    def last_step_ms(self) -> float:
        ms = C.c_double()
        _batch_check(lib().pixvod_batch_last_step_ms(self._h, C.byref(ms)))
        return ms.value

    def track(self, frames, n_iters: int, maps: bool = False, normals=None):
        """One frame per sequence; with `normals` (one normal map per frame)
        sequences whose keyframe test fires are re-anchored on the frame just
        tracked inside the same frame step."""
        keep, ptrs, where = [], [], None
        for f in frames:
            p, w, k = _ptr(f)
            if where is None:
                where = w
            if w != where:
                raise ValueError("all frames must live in the same memory")
            keep.append(k)
            ptrs.append(p)
        nptrs = None
        if normals is not None:
            nptrs = []
            for nm in normals:
                p, w, k = _ptr(nm)
                if w != where:
                    raise ValueError("frames and normals must live in the same memory")
                keep.append(k)
                nptrs.append(p)
        outs = (TrackOut * self.n)()
        maps_out = []
        for i, (H, W) in enumerate(self.shapes):
            outs[i].out_where = HOST
            if maps:
                inv = np.empty((H, W), np.float32)
                var = np.empty((H, W), np.float32)
                outs[i].inv_depth, outs[i].inv_depth_var = inv.ctypes.data, var.ctypes.data
                maps_out.append((inv, var))
            else:
                maps_out.append((None, None))
        self._follow_torch(where)
        if nptrs is None:
            _batch_check(lib().pixvod_batch_track(self._h, (C.c_void_p * self.n)(*ptrs), where, int(n_iters), outs))
        else:
            _batch_check(lib().pixvod_batch_track_reanchor(self._h, (C.c_void_p * self.n)(*ptrs),
                                                           (C.c_void_p * self.n)(*nptrs), where, int(n_iters), outs))
        return [dict(xi=np.array(o.xi_rel[:]), T_world=np.array(o.T_world[:]).reshape(4, 4),
                     valid_fraction=float(o.valid_fraction), frames_since_keyframe=int(o.frames_since_keyframe),
                     flags=int(o.flags), inv_depth=mo[0], inv_depth_var=mo[1])
                for o, mo in zip(outs, maps_out)]

    def get_state(self, seq: int) -> np.ndarray:
        H, W = self.shapes[seq]
        s = np.empty((N_PLANES, H, W), np.float32)
        _batch_check(lib().pixvod_batch_get_state(self._h, int(seq), C.c_void_p(s.ctypes.data), HOST))
        return s

    def set_state(self, seq: int, state: np.ndarray):
        H, W = self.shapes[seq]
        s = np.ascontiguousarray(state, dtype=np.float32)
        if s.shape != (N_PLANES, H, W):
            raise ValueError(f"state must be {(N_PLANES, H, W)}")
        _batch_check(lib().pixvod_batch_set_state(self._h, int(seq), C.c_void_p(s.ctypes.data), HOST))


class Unrolled(_FollowsTorchStream):
    """Differentiable unrolled tracking of target frames against one keyframe.

    forward() runs n_iters GBP iterations per frame from the keyframe's
    initial state and records a checkpoint every ckpt_every iterations on the
    device; backward() runs the hand-written adjoint over that tape and returns
    the gradients of <xi_bar, xi> + <inv_depth_bar, inv_depth> with respect to
    the photometric sigma map, sigma_N and the Huber threshold. A context holds
    the tape of its last forward only.
    """

    def __init__(self, H: int, W: int, K, n_iters: int, max_frames: int, ckpt_every: int = 10,
                 params: Optional[Params] = None, **overrides):
        self.H, self.W = int(H), int(W)
        if params is None:
            params = default_params(**overrides)
        self.params = params
        self.n_iters, self.max_frames = int(n_iters), int(max_frames)
        Kc = Intrinsics(*[float(x) for x in K])
        h = C.c_void_p()
        _batch_check(lib().pixvod_unroll_create(self.H, self.W, C.byref(Kc), C.byref(params), self.max_frames,
                                                self.n_iters, int(ckpt_every), C.byref(h)))
        self._h = h
        self.n_frames = 0

    def close(self):
        if getattr(self, "_h", None):
            lib().pixvod_unroll_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind_stream(self, handle):
        _batch_check(lib().pixvod_unroll_set_stream(self._h, handle))

    def set_keyframe(self, img, normals):
        pi, wi, ki = _ptr(img)
        pn, wn, kn = _ptr(normals)
        if wi != wn:
            raise ValueError("image and normals must live in the same memory")
        self._follow_torch(wi)
        _batch_check(lib().pixvod_unroll_set_keyframe(self._h, C.c_void_p(pi), C.c_void_p(pn), wi))

    def set_state(self, state):
        """The state the forward passes start from, in the exchange layout of
        Tracker.get_state (123 x H x W float32)."""
        ps, ws, ks = _ptr(state)
        self._follow_torch(ws)
        _batch_check(lib().pixvod_unroll_set_state(self._h, C.c_void_p(ps), ws))

    def forward(self, frames, sigma_map, sigma_N: float, huber_k: float, out_device: bool = False):
        """frames (F, H, W) float32; returns xi (F, 6) float64 numpy and the
        inverse-depth maps (F, H, W) float32 (numpy, or a CUDA tensor)."""
        pf, wf, kf = _ptr(frames)
        ps, ws, ks = _ptr(sigma_map)
        F = int(np.prod(frames.shape)) // (self.H * self.W)
        xi = np.zeros((F, 6), np.float64)
        if out_device:
            rho = torch.empty((F, self.H, self.W), dtype=torch.float32, device="cuda")
            pr, wr = rho.data_ptr(), DEVICE
        else:
            rho = np.empty((F, self.H, self.W), np.float32)
            pr, wr = rho.ctypes.data, HOST
        self._follow_torch(wf, ws, wr)
        _batch_check(lib().pixvod_unroll_forward(self._h, C.c_void_p(pf), F, wf, C.c_void_p(ps), ws,
                                                 float(sigma_N), float(huber_k), C.c_void_p(xi.ctypes.data),
                                                 C.c_void_p(pr), wr))
        self.n_frames = F
        return xi, rho

    def backward(self, xi_bar=None, inv_depth_bar=None, grad_device: bool = False):
        """Gradients (sigma map (H, W) float32, sigma_N, huber_k) of the last
        forward for the given output cotangents (None = zero)."""
        xb = None
        if xi_bar is not None:
            xb = np.ascontiguousarray(np.asarray(xi_bar, dtype=np.float64).reshape(self.n_frames, 6))
        pr, wr, kr = (None, HOST, None) if inv_depth_bar is None else _ptr(inv_depth_bar)
        if grad_device:
            g = torch.empty((self.H, self.W), dtype=torch.float32, device="cuda")
            pg, wg = g.data_ptr(), DEVICE
        else:
            g = np.empty((self.H, self.W), np.float32)
            pg, wg = g.ctypes.data, HOST
        gN, gk = C.c_double(), C.c_double()
        self._follow_torch(wr, wg)
        _batch_check(lib().pixvod_unroll_backward(self._h, None if xb is None else C.c_void_p(xb.ctypes.data),
                                                  None if pr is None else C.c_void_p(pr), wr, C.c_void_p(pg), wg,
                                                  C.byref(gN), C.byref(gk)))
        return g, gN.value, gk.value

    def last_ms(self):
        """(forward ms, backward ms) of the last calls, timed with HIP events."""
        f, b = C.c_double(), C.c_double()
        _batch_check(lib().pixvod_unroll_last_ms(self._h, C.byref(f), C.byref(b)))
        return f.value, b.value


class _UnrolledTrack(torch.autograd.Function):
    @staticmethod
    def forward(ctx, unroll, frames, sigma_map, sigma_N, huber_k):
        dev = sigma_map.device
        xi, rho = unroll.forward(frames.detach().contiguous(), sigma_map.detach().to(torch.float32).contiguous(),
                                 float(sigma_N), float(huber_k), out_device=dev.type == "cuda")
        ctx.unroll = unroll
        ctx.meta = (dev, sigma_map.dtype, sigma_N.dtype, huber_k.dtype)
        rho_t = rho if isinstance(rho, torch.Tensor) else torch.from_numpy(rho)
        return torch.from_numpy(xi).to(dev), rho_t

    @staticmethod
    def backward(ctx, xi_bar, rho_bar):
        dev, sdt, ndt, kdt = ctx.meta
        rb = rho_bar.detach().to(torch.float32).contiguous()
        g, gN, gk = ctx.unroll.backward(xi_bar.detach().cpu().numpy(), rb, grad_device=rb.is_cuda)
        g_t = (g if isinstance(g, torch.Tensor) else torch.from_numpy(g)).to(device=dev, dtype=sdt)
        return (None, None, g_t, torch.tensor(gN, dtype=ndt, device=dev), torch.tensor(gk, dtype=kdt, device=dev))


def unrolled_track(unroll: Unrolled, frames, sigma_map, sigma_N, huber_k):
    """torch.autograd entry point: (xi (F, 6) float64, inverse depth (F, H, W))
    as functions of the sigma map (H, W), sigma_N and huber_k (0-d tensors).
    The backward pass is the library's adjoint; one graph per context at a time."""
    return _UnrolledTrack.apply(unroll, frames, sigma_map, sigma_N, huber_k)


class Central(_FollowsTorchStream):
    """Centralised IRLS Gauss-Newton baseline: one global pose and per-pixel
    log-depths, every pixel accessible at once (the normal equations solved by
    FP64 preconditioned conjugate gradients on the GPU)."""

    def __init__(self, H: int, W: int, K, max_cg: int = 500, cg_tol: float = 1e-10,
                 params: Optional[Params] = None, **overrides):
        self.H, self.W = int(H), int(W)
        if params is None:
            params = default_params(**overrides)
        self.params = params
        Kc = Intrinsics(*[float(x) for x in K])
        h = C.c_void_p()
        _check(lib().pixvod_central_create(self.H, self.W, C.byref(Kc), C.byref(params), int(max_cg),
                                           float(cg_tol), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().pixvod_central_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind_stream(self, handle):
        _check(lib().pixvod_central_set_stream(self._h, handle))

    def set_keyframe(self, img, normals):
        pi, wi, ki = _ptr(img)
        pn, wn, kn = _ptr(normals)
        if wi != wn:
            raise ValueError("img and normals must live in the same memory")
        self._follow_torch(wi)
        _check(lib().pixvod_central_set_keyframe(self._h, C.c_void_p(pi), C.c_void_p(pn), wi))

    def set_point(self, xi=None, log_depth=None):
        x = None if xi is None else np.ascontiguousarray(xi, np.float64)
        d = None if log_depth is None else np.ascontiguousarray(log_depth, np.float64).reshape(-1)
        _check(lib().pixvod_central_set_point(self._h, None if x is None else C.c_void_p(x.ctypes.data),
                                              None if d is None else C.c_void_p(d.ctypes.data)))

    def get_point(self):
        xi = np.zeros(6)
        d = np.zeros(self.H * self.W)
        _check(lib().pixvod_central_get_point(self._h, C.c_void_p(xi.ctypes.data), C.c_void_p(d.ctypes.data)))
        return xi, d.reshape(self.H, self.W)

    def track(self, frame, n_iters: int, maps: bool = True, out_device: bool = False):
        pf, wf, kf = _ptr(frame)
        xi = np.zeros(6)
        st = CentralStats()
        inv = None
        pinv = None
        if maps:
            if out_device:
                inv = torch.empty((self.H, self.W), dtype=torch.float32, device="cuda")
                pinv = inv.data_ptr()
            else:
                inv = np.zeros((self.H, self.W), np.float32)
                pinv = inv.ctypes.data
        self._follow_torch(wf, DEVICE if (maps and out_device) else HOST)
        _check(lib().pixvod_central_track(self._h, C.c_void_p(pf), wf, int(n_iters), C.c_void_p(xi.ctypes.data),
                                          None if pinv is None else C.c_void_p(pinv),
                                          DEVICE if out_device else HOST, C.byref(st)))
        return dict(xi=xi, inv_depth=inv, cg_iters=st.cg_iters, last_cg_iters=st.last_cg_iters,
                    last_rel_residual=st.last_rel_residual, valid_fraction=st.valid_fraction, flags=st.flags)

    def last_ms(self) -> float:
        ms = C.c_double()
        _check(lib().pixvod_central_last_ms(self._h, C.byref(ms)))
        return ms.value


def version() -> str:
    return lib().pixvod_version().decode()
