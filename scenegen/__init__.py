"""Seeded synthetic inputs: city scenes, their LoD hierarchy, and walkthroughs.

This module only produces input data (numpy arrays and camera records). It
holds none of the rendering method's arithmetic, and both the FP64 oracle and
the HIP renderer read what it produces. The heavy part (leaf draws and the
hierarchy build for up to 1.8e7 leaves) is plain C in ``vyscene.c``, compiled
with gcc on first use or by ``build_lib()``.

Scene recipe (the three walkthrough workloads):
  * leaves: half on a square ground plane (z = 0), half on the faces of
    box-shaped buildings (footprint U(10, 40) m per side, height U(5, 30) m,
    centres uniform, rejected within 15 m of the walkthrough path);
  * log-scales N(ln 0.3, 0.5) per axis, unit quaternions from normalised
    N(0, I4), opacity logits N(0, 1.5), SH degree 3 with DC ~ N(0.5, 0.2) and
    the other 45 coefficients ~ N(0, 0.2);
  * hierarchy: binary median split on the longest axis, BFS node order,
    moment-matched internal nodes (see vyscene.c).
Camera convention (OpenCV): x_cam = R (x_world - pos), +x right, +y down,
+z forward; pixel (i, j) has its centre at (i + 0.5, j + 0.5).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vyscene.c")
_LIB = os.path.join(_HERE, "libvyscene.so")
_lib = None


def build_lib(force: bool = False) -> str:
    """Compile vyscene.c into libvyscene.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_lib()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.vs_gen_leaves.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int64, P, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      P, P, P, P, P]
        lib.vs_gen_leaves.restype = None
        lib.vs_build_tree.argtypes = [ctypes.c_int64, P, P, P, P, P, P, ctypes.c_int]
        lib.vs_build_tree.restype = ctypes.c_int
        lib.vs_fill_nodes.argtypes = [ctypes.c_int64, ctypes.c_int, P, P, P, P, P, P, P, P,
                                      P, P, P, P, P, P, P, ctypes.c_double]
        lib.vs_fill_nodes.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


# --------------------------------------------------------------------------
# Workload definitions
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class CityConfig:
    name: str
    n_leaf: int
    extent: float          # side of the square ground plane (m)
    n_buildings: int
    frames: int
    width: int
    height: int
    taus: tuple
    speed: tuple           # (min, max) m/frame
    yaw_max_deg: float     # max |yaw rate| in degrees/frame
    fov_x_deg: float = 60.0
    eye: float = 1.7
    scene_seed: int = 1000
    path_seed: int = 2000


CONFIGS = {
    # 2e4 leaves, 256x256, 8 frames, tau = 2 px: small enough for the oracle on every frame.
    "tiny": CityConfig("tiny", 20_000, 200.0, 40, 8, 256, 256, (2.0,), (1.5, 1.5), 1.0,
                       scene_seed=1000, path_seed=2000),
    # 2e6 leaves, 1280x720, 120 frames, tau = 2 px: the plain full-search renderer workload.
    "med": CityConfig("med", 2_000_000, 2000.0, 4000, 120, 1280, 720, (2.0,), (1.5, 1.5), 1.0,
                      scene_seed=1001, path_seed=2001),
    # 1.8e7 leaves, 1920x1080, 300 frames, tau in {1, 2, 4}: the city-scale walkthrough.
    "full": CityConfig("full", 18_000_000, 6000.0, 30000, 300, 1920, 1080, (1.0, 2.0, 4.0), (1.0, 3.0),
                       2.0, scene_seed=1002, path_seed=2002),
}


def scaled_config(base: str, n_leaf: int, **kw) -> CityConfig:
    """A config with the same leaf density as `base` but `n_leaf` leaves."""
    c = CONFIGS[base]
    ratio = n_leaf / c.n_leaf
    d = dict(c.__dict__)
    d.update(name=f"{base}@{n_leaf}", n_leaf=n_leaf, extent=c.extent * math.sqrt(ratio),
             n_buildings=max(1, int(round(c.n_buildings * ratio))))
    d.update(kw)
    return CityConfig(**d)


# --------------------------------------------------------------------------
# Cameras and walkthroughs
# --------------------------------------------------------------------------

@dataclass
class Camera:
    R: np.ndarray          # (3, 3) float32, world -> camera rotation, rows = camera axes
    pos: np.ndarray        # (3,) float32, camera centre in world coordinates
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.2

    def as_f32(self):
        return dict(R=np.asarray(self.R, np.float32), pos=np.asarray(self.pos, np.float32),
                    fx=np.float32(self.fx), fy=np.float32(self.fy), cx=np.float32(self.cx),
                    cy=np.float32(self.cy), width=int(self.width), height=int(self.height),
                    near=np.float32(self.near))


def look_camera(pos, yaw, pitch, width, height, fov_x_deg=60.0, near=0.2) -> Camera:
    """Camera at `pos` (z-up world) looking along heading `yaw` (rad, from +x
    towards +y) tilted by `pitch` (rad, positive = up). All fields are rounded
    to float32 once here; consumers read these float32 values."""
    cy_, sy_ = math.cos(yaw), math.sin(yaw)
    cp, sp = math.cos(pitch), math.sin(pitch)
    fwd = np.array([cy_ * cp, sy_ * cp, sp])
    right = np.array([sy_, -cy_, 0.0])
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd]).astype(np.float32)
    f = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(R=R, pos=np.asarray(pos, np.float32), fx=float(np.float32(f)), fy=float(np.float32(f)),
                  cx=width / 2.0, cy=height / 2.0, width=width, height=height, near=float(np.float32(near)))


def walkthrough_path(cfg: CityConfig, seed: int | None = None, frames: int | None = None):
    """Smooth street-level path: positions (frames, 3) and headings (frames,).

    Speed and yaw rate are sinusoids of seeded phase: speed within cfg.speed,
    |yaw rate| <= cfg.yaw_max_deg per frame. Starts near the plane centre."""
    seed = cfg.path_seed if seed is None else seed
    frames = cfg.frames if frames is None else frames
    rng = np.random.default_rng(seed)
    ph_v, ph_y, yaw0 = rng.uniform(0, 2 * math.pi, 3)
    per_v, per_y = rng.uniform(60, 140, 2)
    x0 = rng.uniform(-0.02, 0.02, 2) * cfg.extent
    smin, smax = cfg.speed
    pos = np.zeros((frames, 3))
    yaw = np.zeros(frames)
    p = np.array([x0[0], x0[1]])
    h = yaw0
    for t in range(frames):
        pos[t, :2] = p
        pos[t, 2] = cfg.eye
        yaw[t] = h
        v = 0.5 * (smin + smax) + 0.5 * (smax - smin) * math.sin(2 * math.pi * t / per_v + ph_v)
        h = h + math.radians(cfg.yaw_max_deg) * math.sin(2 * math.pi * t / per_y + ph_y)
        p = p + v * np.array([math.cos(h), math.sin(h)])
    return pos, yaw


def walkthrough(cfg: CityConfig, seed: int | None = None, frames: int | None = None,
                width: int | None = None, height: int | None = None, pitch_deg: float = 0.0):
    pos, yaw = walkthrough_path(cfg, seed, frames)
    W = cfg.width if width is None else width
    H = cfg.height if height is None else height
    return [look_camera(pos[t], yaw[t], math.radians(pitch_deg), W, H, cfg.fov_x_deg)
            for t in range(len(yaw))]


# --------------------------------------------------------------------------
# Scenes
# --------------------------------------------------------------------------

@dataclass
class Scene:
    """Node arrays of the LoD hierarchy in BFS order (node 0 is the root).

    Children of node n are first_child[n] .. first_child[n] + child_count[n] - 1
    (contiguous); leaves have first_child = -1 and child_count = 0."""
    n_leaf: int
    parent: np.ndarray        # (N,) int32, -1 at the root
    first_child: np.ndarray   # (N,) int32
    child_count: np.ndarray   # (N,) int32
    aabb_lo: np.ndarray       # (N, 3) float32
    aabb_hi: np.ndarray       # (N, 3) float32
    mean: np.ndarray          # (N, 3) float32
    log_scale: np.ndarray     # (N, 3) float32
    quat: np.ndarray          # (N, 4) float32 (w, x, y, z), unit
    opacity_logit: np.ndarray  # (N,) float32
    sh: np.ndarray            # (N, 16, 3) float32, index l*l + l + m, channel
    level_start: np.ndarray = field(default=None)  # first node id of every BFS level (+ end)

    @property
    def n_nodes(self) -> int:
        return int(self.parent.shape[0])


def place_buildings(cfg: CityConfig, path_xy: np.ndarray, seed: int) -> np.ndarray:
    """(n_b, 5) float64 rows (cx, cy, half_x, half_y, height), rejected within
    15 m (plus the footprint half-diagonal) of any walkthrough path point."""
    rng = np.random.default_rng(seed + 7919)
    out = []
    need = cfg.n_buildings
    tries = 0
    while need > 0 and tries < 50:
        m = max(64, int(need * 1.5))
        c = rng.uniform(-0.5, 0.5, (m, 2)) * cfg.extent
        hs = rng.uniform(5.0, 20.0, (m, 2))
        h = rng.uniform(5.0, 30.0, m)
        r = 15.0 + np.hypot(hs[:, 0], hs[:, 1])
        ok = np.ones(m, bool)
        if len(path_xy):
            for s in range(0, len(path_xy), 64):
                P = path_xy[s:s + 64]
                d = np.min(np.hypot(c[:, None, 0] - P[None, :, 0], c[:, None, 1] - P[None, :, 1]), axis=1)
                ok &= d > r
        sel = np.nonzero(ok)[0][:need]
        out.append(np.concatenate([c[sel], hs[sel], h[sel, None]], axis=1))
        need -= len(sel)
        tries += 1
    return np.ascontiguousarray(np.concatenate(out, axis=0)[:cfg.n_buildings], dtype=np.float64)


def generate_leaves(cfg: CityConfig, seed: int | None = None, path_xy: np.ndarray | None = None):
    seed = cfg.scene_seed if seed is None else seed
    if path_xy is None:
        pos, _ = walkthrough_path(cfg)
        path_xy = pos[:, :2]
    B = place_buildings(cfg, path_xy, seed)
    n = cfg.n_leaf
    mean = np.empty((n, 3), np.float32)
    ls = np.empty((n, 3), np.float32)
    q = np.empty((n, 4), np.float32)
    lg = np.empty((n,), np.float32)
    sh = np.empty((n, 16, 3), np.float32)
    _load().vs_gen_leaves(seed, n, cfg.extent, 0.5, B.shape[0], _p(B), math.log(0.3), 0.5, 1.5, 0.5, 0.2,
                          _p(mean), _p(ls), _p(q), _p(lg), _p(sh))
    return dict(mean=mean, log_scale=ls, quat=q, opacity_logit=lg, sh=sh, buildings=B)


def build_hierarchy(leaves: dict, logit_clamp: float = 30.0) -> Scene:
    """Median-split binary hierarchy over the leaves (see module docstring)."""
    lib = _load()
    n = int(leaves["mean"].shape[0])
    N = 2 * n - 1
    parent = np.empty(N, np.int32)
    first_child = np.empty(N, np.int32)
    child_count = np.empty(N, np.int32)
    leaf_of = np.empty(N, np.int32)
    level_start = np.zeros(80, np.int64)
    nlev = lib.vs_build_tree(n, _p(leaves["mean"]), _p(parent), _p(first_child), _p(child_count),
                             _p(leaf_of), _p(level_start), 79)
    if nlev < 0:
        raise RuntimeError(f"vs_build_tree failed ({nlev})")
    mean = np.empty((N, 3), np.float32)
    ls = np.empty((N, 3), np.float32)
    q = np.empty((N, 4), np.float32)
    lg = np.empty((N,), np.float32)
    sh = np.empty((N, 16, 3), np.float32)
    lo = np.empty((N, 3), np.float32)
    hi = np.empty((N, 3), np.float32)
    rc = lib.vs_fill_nodes(n, nlev, _p(level_start), _p(first_child), _p(leaf_of),
                           _p(leaves["mean"]), _p(leaves["log_scale"]), _p(leaves["quat"]),
                           _p(leaves["opacity_logit"]), _p(leaves["sh"]),
                           _p(mean), _p(ls), _p(q), _p(lg), _p(sh), _p(lo), _p(hi), logit_clamp)
    if rc != 0:
        raise RuntimeError(f"vs_fill_nodes failed ({rc})")
    return Scene(n_leaf=n, parent=parent, first_child=first_child, child_count=child_count,
                 aabb_lo=lo, aabb_hi=hi, mean=mean, log_scale=ls, quat=q, opacity_logit=lg, sh=sh,
                 level_start=level_start[:nlev + 1].copy())


def make_city(cfg: CityConfig | str, seed: int | None = None) -> Scene:
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    return build_hierarchy(generate_leaves(cfg, seed))


def tree_from_arrays(parent, first_child, child_count, aabb_lo, aabb_hi, mean=None, log_scale=None,
                     quat=None, opacity_logit=None, sh=None) -> Scene:
    """Wrap hand-built node arrays (tests) as a Scene; missing Gaussian
    attributes get neutral defaults."""
    N = len(parent)
    f32 = lambda a, shape, v: (np.full(shape, v, np.float32) if a is None
                               else np.ascontiguousarray(a, np.float32).reshape(shape))
    qd = np.zeros((N, 4), np.float32)
    qd[:, 0] = 1
    return Scene(n_leaf=int(np.sum(np.asarray(child_count) == 0)),
                 parent=np.ascontiguousarray(parent, np.int32),
                 first_child=np.ascontiguousarray(first_child, np.int32),
                 child_count=np.ascontiguousarray(child_count, np.int32),
                 aabb_lo=f32(aabb_lo, (N, 3), 0), aabb_hi=f32(aabb_hi, (N, 3), 0),
                 mean=f32(mean, (N, 3), 0), log_scale=f32(log_scale, (N, 3), math.log(0.3)),
                 quat=qd if quat is None else f32(quat, (N, 4), 0),
                 opacity_logit=f32(opacity_logit, (N,), 0), sh=f32(sh, (N, 16, 3), 0))


def random_gaussians(n: int, seed: int, width: int, height: int, depth_range=(2.0, 30.0),
                     scale_range=(-3.0, 0.0)) -> Scene:
    """Flat list of n Gaussians (a one-level 'hierarchy' is not built) placed in
    front of the identity camera, for splatting tests: returns a Scene whose
    node arrays hold the Gaussians; tree fields are leaves with parent -1."""
    rng = np.random.default_rng(seed)
    f = (width / 2.0) / math.tan(math.radians(30.0))
    z = rng.uniform(*depth_range, n)
    u = rng.uniform(-0.1 * width, 1.1 * width, n)
    v = rng.uniform(-0.1 * height, 1.1 * height, n)
    x = (u - width / 2) * z / f
    y = (v - height / 2) * z / f
    mean = np.stack([x, y, z], 1).astype(np.float32)
    ls = rng.uniform(*scale_range, (n, 3)).astype(np.float32)
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    lg = rng.normal(0, 1.5, n).astype(np.float32)
    sh = rng.normal(0, 0.2, (n, 16, 3)).astype(np.float32)
    sh[:, 0, :] += 0.5
    neg = -np.ones(n, np.int32)
    return Scene(n_leaf=n, parent=neg, first_child=neg.copy(), child_count=np.zeros(n, np.int32),
                 aabb_lo=mean - 1, aabb_hi=mean + 1, mean=mean, log_scale=ls, quat=q.astype(np.float32),
                 opacity_logit=lg, sh=sh)


def identity_camera(width: int, height: int, fov_x_deg: float = 60.0) -> Camera:
    f = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(R=np.eye(3, dtype=np.float32), pos=np.zeros(3, np.float32), fx=float(np.float32(f)),
                  fy=float(np.float32(f)), cx=width / 2.0, cy=height / 2.0, width=width, height=height)
