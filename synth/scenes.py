"""Piecewise-planar textured scenes, camera trajectories and a ray-casting renderer.

Conventions used by every consumer of these inputs:

* pinhole camera, pixel centres at integer coordinates (u, v), u in [0, W),
  v in [0, H); x right, y down, z forward;
* a camera pose is the 4x4 matrix T_wc mapping camera coordinates to world
  coordinates; frame 0 of every sequence is the world frame (T_wc = I);
* images are float32 intensities, depth is the camera z-depth (float64),
  normals are unit float32 3-vectors in the rendering camera's frame.

Textures are seeded value noise evaluated through an integer hash of the
lattice coordinates, so any region of any plane has a deterministic texture
without storing lattices. All randomness comes from numpy's PCG64 generator
seeded by the caller.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np
from scipy.spatial.transform import Rotation

_U64 = np.uint64


@dataclasses.dataclass(frozen=True)
class Camera:
    H: int
    W: int
    fx: float
    fy: float
    cx: float
    cy: float

    @staticmethod
    def default(H: int, W: int) -> "Camera":
        """Intrinsics with a 56.1 degree horizontal field of view (f = 30 W / 32)
        and the principal point at (W/2, H/2)."""
        f = 30.0 * W / 32.0
        return Camera(H, W, f, f, W / 2.0, H / 2.0)


@dataclasses.dataclass
class Plane:
    center: np.ndarray          # (3,) world point on the plane
    normal: np.ndarray          # (3,) unit normal
    axis1: np.ndarray           # (3,) unit in-plane axis
    axis2: np.ndarray           # (3,) unit in-plane axis, axis1 x axis2 = normal
    half1: float                # half extent along axis1 (inf = unbounded)
    half2: float
    lattice: float              # base lattice spacing of the texture, metres
    octaves: int = 1
    persistence: float = 0.5
    tex_seed: int = 0


@dataclasses.dataclass
class Scene:
    planes: List[Plane]


# ----------------------------------------------------------------------------
# hashed value noise


def _splitmix64(x: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = x + _U64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> _U64(30))) * _U64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> _U64(27))) * _U64(0x94D049BB133111EB)
        return z ^ (z >> _U64(31))


def _lattice_value(seed: int, octave: int, ix: np.ndarray, iy: np.ndarray) -> np.ndarray:
    """Deterministic U[0,1) value for integer lattice points (ix, iy)."""
    with np.errstate(over="ignore"):
        k = _splitmix64(np.full(ix.shape, seed * 1000003 + octave, dtype=np.uint64))
        k = _splitmix64(k ^ ix.astype(np.int64).view(np.uint64))
        k = _splitmix64(k ^ (iy.astype(np.int64).view(np.uint64) * _U64(0x632BE59BD9B4E019)))
    return (k >> _U64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _smoothstep(t: np.ndarray) -> np.ndarray:
    return t * t * (3.0 - 2.0 * t)


def value_noise_texture(x: np.ndarray, y: np.ndarray, seed: int, octaves: int = 1,
                        persistence: float = 0.5) -> np.ndarray:
    """Multi-octave value noise at continuous lattice coordinates (x, y).

    Octave k has lattice spacing 2^-k of the base and amplitude persistence^k;
    the sum is divided by the total amplitude so values stay in [0, 1].
    """
    out = np.zeros(np.broadcast(x, y).shape, dtype=np.float64)
    amp, total = 1.0, 0.0
    for k in range(octaves):
        s = float(2 ** k)
        xs, ys = x * s, y * s
        ix, iy = np.floor(xs), np.floor(ys)
        fx, fy = _smoothstep(xs - ix), _smoothstep(ys - iy)
        ix, iy = ix.astype(np.int64), iy.astype(np.int64)
        v00 = _lattice_value(seed, k, ix, iy)
        v10 = _lattice_value(seed, k, ix + 1, iy)
        v01 = _lattice_value(seed, k, ix, iy + 1)
        v11 = _lattice_value(seed, k, ix + 1, iy + 1)
        out += amp * ((v00 * (1 - fx) + v10 * fx) * (1 - fy) + (v01 * (1 - fx) + v11 * fx) * fy)
        total += amp
        amp *= persistence
    return out / total


# ----------------------------------------------------------------------------
# rendering


def so3_exp(rotvec: Sequence[float]) -> np.ndarray:
    """Rotation matrix of a rotation vector (scene construction only)."""
    return Rotation.from_rotvec(np.asarray(rotvec, dtype=np.float64)).as_matrix()


def pose_from_motion(rotvec: Sequence[float], position: Sequence[float]) -> np.ndarray:
    T = np.eye(4)
    T[:3, :3] = so3_exp(rotvec)
    T[:3, 3] = np.asarray(position, dtype=np.float64)
    return T


def render(scene: Scene, cam: Camera, T_wc: np.ndarray):
    """Ray-cast the scene from camera pose T_wc.

    Returns (image float32 HxW, z-depth float64 HxW, normals float32 HxWx3 in
    the camera frame, plane index int32 HxW with -1 where nothing is hit).
    Pixels that hit nothing get intensity 0.5, depth inf and normal (0,0,-1).
    """
    H, W = cam.H, cam.W
    u, v = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    q = np.stack([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy, np.ones_like(u)], axis=-1)
    R, o = T_wc[:3, :3], T_wc[:3, 3]
    d = q @ R.T                                    # world ray directions (z-depth scale)
    best = np.full((H, W), np.inf)
    idx = np.full((H, W), -1, dtype=np.int32)
    s1 = np.zeros((H, W))
    s2 = np.zeros((H, W))
    for k, pl in enumerate(scene.planes):
        denom = d @ pl.normal
        with np.errstate(divide="ignore", invalid="ignore"):
            lam = np.dot(pl.center - o, pl.normal) / denom
        X = o + lam[..., None] * d
        rel = X - pl.center
        c1, c2 = rel @ pl.axis1, rel @ pl.axis2
        hit = (np.abs(denom) > 1e-12) & (lam > 1e-6) & (lam < best)
        hit &= (np.abs(c1) <= pl.half1) & (np.abs(c2) <= pl.half2)
        best = np.where(hit, lam, best)
        idx = np.where(hit, k, idx)
        s1 = np.where(hit, c1, s1)
        s2 = np.where(hit, c2, s2)
    img = np.full((H, W), 0.5)
    nrm = np.zeros((H, W, 3))
    nrm[..., 2] = -1.0
    for k, pl in enumerate(scene.planes):
        m = idx == k
        if not np.any(m):
            continue
        img[m] = value_noise_texture(s1[m] / pl.lattice, s2[m] / pl.lattice, pl.tex_seed,
                                     pl.octaves, pl.persistence)
        n_c = R.T @ pl.normal
        if n_c[2] > 0:          # orient towards the camera; the sign carries no information
            n_c = -n_c
        nrm[m] = n_c
    return img.astype(np.float32), best, nrm.astype(np.float32), idx


# ----------------------------------------------------------------------------
# the tiny image pair


def tiny_pair(seed: int = 0, H: int = 24, W: int = 32, inv_depth: float = 0.5,
              move_x: float = 0.01, yaw_deg: float = 0.5, lattice_px: float = 4.0,
              rotvec=None, trans=None, principal=None):
    """Textured fronto-parallel plane seen by a keyframe camera at the origin and
    by a target camera moved by `move_x` metres along x and yawed by `yaw_deg`
    degrees about its y axis (fx = fy = 30 W/32, principal point (W/2, H/2)).

    `rotvec` / `trans` (camera rotation vector and position of the target
    camera in the keyframe frame) override the x-move and yaw when given;
    `principal` overrides the principal point (cx, cy).

    Returns a dict with the camera, source/target images, keyframe depth and
    normals, and T_ts = T_{target<-source}, the transform that maps keyframe
    camera points into the target camera.
    """
    cam = Camera.default(H, W)
    if principal is not None:
        cam = Camera(H, W, cam.fx, cam.fy, float(principal[0]), float(principal[1]))
    z = 1.0 / inv_depth
    lattice = lattice_px * z / cam.fx
    plane = Plane(center=np.array([0.0, 0.0, z]), normal=np.array([0.0, 0.0, -1.0]),
                  axis1=np.array([1.0, 0.0, 0.0]), axis2=np.array([0.0, -1.0, 0.0]),
                  half1=math.inf, half2=math.inf, lattice=lattice, octaves=1,
                  tex_seed=seed * 7919 + 17)
    scene = Scene([plane])
    T_src = np.eye(4)
    rv = [0.0, math.radians(yaw_deg), 0.0] if rotvec is None else rotvec
    tr = [move_x, 0.0, 0.0] if trans is None else trans
    T_tgt = pose_from_motion(rv, tr)
    I_s, D_s, N_s, _ = render(scene, cam, T_src)
    I_t, _, _, _ = render(scene, cam, T_tgt)
    T_ts = np.linalg.inv(T_tgt) @ T_src
    return dict(cam=cam, I_s=I_s, I_t=I_t, depth_s=D_s, normals_s=N_s, T_ts=T_ts,
                scene=scene, T_src=T_src, T_tgt=T_tgt)


# ----------------------------------------------------------------------------
# sequences of piecewise-planar scenes


@dataclasses.dataclass(frozen=True)
class SequenceConfig:
    name: str
    H: int
    W: int
    n_frames: int
    n_planes: int
    inv_depth_range: Tuple[float, float]
    noise_sigma: float
    occlusion_frac: float
    max_step_t: float           # metres per frame
    max_step_r_deg: float       # degrees per frame
    octaves: int = 4
    lattice_px: float = 4.0
    seed: int = 0


SEQUENCE_CONFIGS = {
    "ppa256": SequenceConfig("ppa256", 256, 256, 100, 6, (0.2, 2.0), 0.01, 0.0, 0.02, 1.0, seed=1),
    "vga": SequenceConfig("vga", 480, 640, 300, 12, (0.2, 2.0), 0.02, 0.10, 0.02, 1.0, seed=2),
    "diff320": SequenceConfig("diff320", 240, 320, 30, 6, (0.2, 2.0), 0.01, 0.0, 0.01, 0.5, seed=3),
}

_BATCH_CLASSES = [(96, 128), (256, 256), (240, 320), (480, 640)]


def batch_resolution(s: int) -> Tuple[int, int]:
    """(H, W) of sequence s of the mixed-resolution batch."""
    return _BATCH_CLASSES[s % 4]


def batch_sequence_config(s: int, n_frames: int = 50, base_seed: int = 1000) -> SequenceConfig:
    H, W = batch_resolution(s)
    return SequenceConfig(f"batch{s}", H, W, n_frames, 6, (0.2, 2.0), 0.01, 0.0, 0.02, 1.0,
                          seed=base_seed + s)


def _orthonormal_axes(n: np.ndarray, angle: float):
    a = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(n, a)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(n, e1)
    c, s = math.cos(angle), math.sin(angle)
    return c * e1 + s * e2, -s * e1 + c * e2


def make_sequence_scene(cfg: SequenceConfig) -> Tuple[Scene, Camera]:
    """Random planes in front of the frame-0 camera plus a fronto-parallel
    background at inverse depth 0.2.

    Plane centres sit on the rays of uniformly drawn pixels at an inverse depth
    drawn from cfg.inv_depth_range; normals lie within 60 degrees of the
    optical axis; half extents are 0.2-1.0 times the plane's depth. Each plane's
    texture has a base lattice of cfg.lattice_px pixels at its own depth.
    """
    rng = np.random.default_rng(cfg.seed)
    cam = Camera.default(cfg.H, cfg.W)
    planes: List[Plane] = []
    zb = 1.0 / 0.2
    planes.append(Plane(center=np.array([0.0, 0.0, zb]), normal=np.array([0.0, 0.0, -1.0]),
                        axis1=np.array([1.0, 0.0, 0.0]), axis2=np.array([0.0, -1.0, 0.0]),
                        half1=math.inf, half2=math.inf,
                        lattice=cfg.lattice_px * zb / cam.fx, octaves=cfg.octaves,
                        tex_seed=cfg.seed * 131 + 1))
    for k in range(cfg.n_planes):
        u = rng.uniform(0.1 * cfg.W, 0.9 * cfg.W)
        v = rng.uniform(0.1 * cfg.H, 0.9 * cfg.H)
        rho = rng.uniform(*cfg.inv_depth_range)
        z = 1.0 / rho
        center = np.array([(u - cam.cx) / cam.fx * z, (v - cam.cy) / cam.fy * z, z])
        tilt = math.acos(rng.uniform(math.cos(math.radians(60.0)), 1.0))
        az = rng.uniform(0.0, 2.0 * math.pi)
        n = np.array([math.sin(tilt) * math.cos(az), math.sin(tilt) * math.sin(az), -math.cos(tilt)])
        a1, a2 = _orthonormal_axes(n, rng.uniform(0.0, math.pi))
        h1 = rng.uniform(0.2, 1.0) * z
        h2 = rng.uniform(0.2, 1.0) * z
        planes.append(Plane(center=center, normal=n, axis1=a1, axis2=a2, half1=h1, half2=h2,
                            lattice=cfg.lattice_px * z / cam.fx, octaves=cfg.octaves,
                            tex_seed=cfg.seed * 131 + 2 + k))
    return Scene(planes), cam


def sequence_poses(cfg: SequenceConfig) -> np.ndarray:
    """Camera poses T_wc for every frame (n_frames x 4 x 4), frame 0 = identity.

    Each of the six motion axes is a sinusoid with a random period in [40, 120]
    frames and a random phase, offset so that it starts at zero; amplitudes are
    scaled so the per-frame translation stays below cfg.max_step_t and the
    per-frame rotation below cfg.max_step_r_deg.
    """
    rng = np.random.default_rng(cfg.seed + 7777)
    periods = rng.uniform(40.0, 120.0, size=6)
    phases = rng.uniform(0.0, 2.0 * math.pi, size=6)
    scale = rng.uniform(0.5, 1.0, size=6)
    bound = np.array([math.radians(cfg.max_step_r_deg)] * 3 + [cfg.max_step_t] * 3)
    amps = 0.9 * bound / math.sqrt(3.0) * periods / (2.0 * math.pi) * scale
    f = np.arange(cfg.n_frames, dtype=np.float64)[:, None]
    x = amps * (np.sin(2.0 * math.pi * f / periods + phases) - np.sin(phases))
    return np.stack([pose_from_motion(x[i, :3], x[i, 3:]) for i in range(cfg.n_frames)])


def _occluder_patches(rng: np.random.Generator, H: int, W: int, frac: float, n: int = 5):
    weights = rng.uniform(0.5, 1.5, size=n)
    areas = frac * H * W * weights / weights.sum()
    out = []
    for k in range(n):
        aspect = rng.uniform(0.5, 2.0)
        w = max(1, int(round(math.sqrt(areas[k] * aspect))))
        h = max(1, int(round(areas[k] / w)))
        w, h = min(w, W), min(h, H)
        x0 = int(rng.integers(0, W - w + 1))
        y0 = int(rng.integers(0, H - h + 1))
        out.append((x0, y0, w, h, int(rng.integers(0, 2 ** 31))))
    return out


def render_sequence_frame(cfg: SequenceConfig, scene: Scene, cam: Camera, poses: np.ndarray,
                          f: int, keyframe: bool = False):
    """Render frame f: returns (image float32, depth, normals, plane index).

    Adds i.i.d. Gaussian noise of cfg.noise_sigma (not clipped). Target frames
    (keyframe=False) of configurations with occlusion get five textured
    rectangles pasted over cfg.occlusion_frac of the image area.
    """
    img, depth, nrm, idx = render(scene, cam, poses[f])
    rng = np.random.default_rng([cfg.seed, f, 1 if keyframe else 0])
    img = img.astype(np.float64)
    if cfg.occlusion_frac > 0 and not keyframe:
        for (x0, y0, w, h, s) in _occluder_patches(rng, cam.H, cam.W, cfg.occlusion_frac):
            yy, xx = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64),
                                 indexing="ij")
            img[y0:y0 + h, x0:x0 + w] = value_noise_texture(xx / 4.0, yy / 4.0, s, 2, 0.5)
    if cfg.noise_sigma > 0:
        img = img + rng.normal(0.0, cfg.noise_sigma, size=img.shape)
    return img.astype(np.float32), depth, nrm, idx
