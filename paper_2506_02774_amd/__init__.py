"""Voyager on MI355X: Python binding of the C-ABI library ``libvoyager.so``.

Argument marshalling only: every step of the per-frame path (LoD cut,
projection, binning, sorting, blending) runs in the library's HIP kernels.
PyTorch provides device memory (tensors) and the HIP stream. There is no CPU
fallback: importing the binding raises if the library has not been built, and
every call raises ``VoyagerError`` on a non-zero status.

The function names follow the C ABI in include/vy.h (vy_scene_upload,
vy_lod_cut, vy_render, ...); ``Scene``, ``Cut`` and ``RenderContext`` are small
owners that keep the device buffers alive for the handles that borrow them.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvoyager.so")

VY_OK, VY_ERR_ARG, VY_ERR_HIP, VY_ERR_CAPACITY, VY_ERR_STATE, VY_ERR_DEVICE = 0, -1, -2, -3, -4, -5
VY_CUT_FRONTIER, VY_CUT_FLAT, VY_CUT_DFS, VY_CUT_CHUNKED = 0, 1, 2, 4
VY_WALK_FULL_EACH = 256
STAGES = ["lod_setup", "lod_flat", "lod_classify", "lod_traverse", "lod_compact", "render_setup", "project",
          "depth_sort", "pair_scan", "emit", "tile_sort", "ranges", "blend_plan", "blend", "bwd_blend", "bwd_project"]


class VoyagerError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class vy_camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("pos", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("znear", ctypes.c_float)]


class vy_view(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_void_p), ("cut", ctypes.c_void_p), ("cam", vy_camera), ("image", ctypes.c_void_p)]


class vy_scene_desc(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64)] + [(k, ctypes.c_void_p) for k in (
        "parent", "first_child", "child_count", "aabb_lo", "aabb_hi", "mean", "log_scale", "quat",
        "opacity_logit", "sh")]


class vy_render_opts(ctypes.Structure):
    _fields_ = [("alpha_filter", ctypes.c_int32), ("bg", ctypes.c_float * 3), ("save_state", ctypes.c_int32),
                ("split_min_pairs", ctypes.c_int32), ("walk", ctypes.c_int32), ("lut_entries", ctypes.c_int32),
                ("band_jobs", ctypes.c_int32)]


class vy_grads(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("mean", "log_scale", "quat", "opacity_logit", "sh", "mean2d",
                                               "quat_raw")]


class vy_session(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("tau", ctypes.c_float), ("alpha_filter", ctypes.c_int32), ("max_gaussians", ctypes.c_int64),
                ("max_pairs", ctypes.c_int64)]


class vy_frame_req(ctypes.Structure):
    _fields_ = [("session", ctypes.c_int32), ("reserved", ctypes.c_int32), ("t_arrival", ctypes.c_double),
                ("cam", vy_camera), ("image", ctypes.c_void_p)]


class vy_frame_stats(ctypes.Structure):
    _fields_ = [("image_hash", ctypes.c_uint64), ("n_cut", ctypes.c_uint32), ("n_pairs", ctypes.c_uint32),
                ("n_visible", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("n_frontier", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class vy_frame_result(ctypes.Structure):
    _fields_ = [("t_admit", ctypes.c_double), ("t_dispatch", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("status", ctypes.c_int32), ("stream", ctypes.c_int32)]


class vy_server_config(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_void_p), ("n_streams", ctypes.c_int32), ("streams", ctypes.POINTER(ctypes.c_void_p)),
                ("max_inflight", ctypes.c_int32), ("max_viewers", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("batch_gaussians", ctypes.c_int64), ("batch_pairs", ctypes.c_int64)]


VY_RUN_REALTIME = 1

_lib = None


def lib():
    """Load libvoyager.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2506_02774_amd.build.build() "
                          "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32, F32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_size_t
    sig = {
        "vy_last_error": ([], ctypes.c_char_p),
        "vy_version": ([], ctypes.c_char_p),
        "vy_scene_workspace_bytes": ([I64], SZ),
        "vy_scene_upload": ([ctypes.POINTER(vy_scene_desc), P, SZ, P, ctypes.POINTER(P)], ctypes.c_int),
        "vy_scene_validate": ([P, ctypes.POINTER(I64), P], ctypes.c_int),
        "vy_scene_update_gaussians": ([P, P, P, P, P, P, P], ctypes.c_int),
        "vy_scene_partition_bytes": ([I64], SZ),
        "vy_scene_partition": ([P, P, SZ, P], ctypes.c_int),
        "vy_partition_plan": ([I64, P, P, P, P, P, ctypes.POINTER(I64), P, P, P, ctypes.POINTER(I64)], ctypes.c_int),
        "vy_scene_num_nodes": ([P], I64),
        "vy_scene_free": ([P], ctypes.c_int),
        "vy_cut_workspace_bytes": ([I64], SZ),
        "vy_cut_create": ([P, P, SZ, ctypes.POINTER(P)], ctypes.c_int),
        "vy_cut_free": ([P], ctypes.c_int),
        "vy_lod_cut": ([P, ctypes.POINTER(vy_camera), F32, P, P, ctypes.c_int, P], ctypes.c_int),
        "vy_cut_counts": ([P, ctypes.POINTER(I64), ctypes.POINTER(I64), P], ctypes.c_int),
        "vy_cut_arrays": ([P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P)], ctypes.c_int),
        "vy_cut_set_frontier": ([P, P, I64, P], ctypes.c_int),
        "vy_render_workspace_bytes": ([I64, I32, I32, I64], SZ),
        "vy_render_ctx_create": ([I64, I32, I32, I64, P, SZ, ctypes.POINTER(P)], ctypes.c_int),
        "vy_render_ctx_free": ([P], ctypes.c_int),
        "vy_render": ([P, P, ctypes.POINTER(vy_camera), ctypes.POINTER(vy_render_opts), P, P, P], ctypes.c_int),
        "vy_render_noalloc": ([P, P, ctypes.POINTER(vy_camera), ctypes.POINTER(vy_render_opts), P, P, P],
                              ctypes.c_int),
        "vy_render_status": ([P, ctypes.POINTER(I64), ctypes.POINTER(I64), P], ctypes.c_int),
        "vy_batch_workspace_bytes": ([I32, I64, I64, I64], SZ),
        "vy_batch_ctx_create": ([I32, I64, I64, I64, P, SZ, ctypes.POINTER(P)], ctypes.c_int),
        "vy_batch_ctx_free": ([P], ctypes.c_int),
        "vy_render_batch": ([ctypes.POINTER(vy_view), I32, ctypes.POINTER(vy_render_opts), P, P], ctypes.c_int),
        "vy_batch_status": ([P, ctypes.POINTER(I64), ctypes.POINTER(I64), P], ctypes.c_int),
        "vy_render_backward": ([P, P, ctypes.POINTER(vy_camera), P, ctypes.POINTER(vy_grads), P, P], ctypes.c_int),
        "vy_render_saved": ([P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                             ctypes.POINTER(P)],
                            ctypes.c_int),
        "vy_render_pairs": ([P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P)], ctypes.c_int),
        "vy_render_projected": ([P] + [ctypes.POINTER(P)] * 4, ctypes.c_int),
        "vy_profile_begin": ([I64], ctypes.c_int),
        "vy_profile_end": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)], ctypes.c_int),
        "vy_stage_name": ([ctypes.c_int], ctypes.c_char_p),
        "vy_measure_peaks_bytes": ([], SZ),
        "vy_measure_peaks": ([P, SZ, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), P],
                             ctypes.c_int),
        # vy_serve.h
        "vy_arena_create": ([P, SZ, ctypes.POINTER(P)], ctypes.c_int),
        "vy_arena_free": ([P], ctypes.c_int),
        "vy_arena_alloc": ([P, SZ, ctypes.POINTER(P)], ctypes.c_int),
        "vy_arena_release": ([P, P], ctypes.c_int),
        "vy_arena_stats": ([P, ctypes.POINTER(SZ), ctypes.POINTER(SZ), ctypes.POINTER(I64), ctypes.POINTER(I64)],
                           ctypes.c_int),
        "vy_session_bytes": ([ctypes.POINTER(vy_session)], SZ),
        "vy_server_create": ([ctypes.POINTER(vy_server_config), ctypes.POINTER(P)], ctypes.c_int),
        "vy_server_free": ([P], ctypes.c_int),
        "vy_server_run": ([P, ctypes.POINTER(vy_session), I32, ctypes.POINTER(vy_frame_req), I64, I32, P,
                           ctypes.POINTER(vy_frame_result)], ctypes.c_int),
        "vy_server_last_run": ([P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(SZ),
                                ctypes.POINTER(I64), ctypes.POINTER(I64)], ctypes.c_int),
        "vy_server_simulate": ([ctypes.POINTER(vy_server_config), ctypes.POINTER(I64), ctypes.POINTER(I64), I32,
                                ctypes.POINTER(vy_frame_req), I64, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_uint32), I32, ctypes.POINTER(vy_frame_result),
                                ctypes.POINTER(I64)], ctypes.c_int),
        "vy_walkthrough": ([P, ctypes.POINTER(vy_camera), I64, F32, I32, ctypes.POINTER(vy_render_opts), P, I32,
                            ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), I64, P,
                            ctypes.POINTER(F32), P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(rc, what=""):
    if rc != VY_OK:
        msg = lib().vy_last_error().decode(errors="replace")
        raise VoyagerError(rc, f"{what}: {msg}" if what else msg)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_camera(cam) -> vy_camera:
    """vy_camera from any object with R, pos, fx, fy, cx, cy, width, height, near."""
    c = vy_camera()
    R = np.asarray(cam.R, np.float32).reshape(9)
    for i in range(9):
        c.R[i] = float(R[i])
    p = np.asarray(cam.pos, np.float32)
    for i in range(3):
        c.pos[i] = float(p[i])
    c.fx, c.fy, c.cx, c.cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    c.width, c.height = int(cam.width), int(cam.height)
    c.znear = float(np.float32(getattr(cam, "near", 0.2)))
    return c


def make_cameras(cams):
    """A ctypes array of vy_camera for a sequence of cameras, the fields of each
    as make_camera() sets them (float32 rounding, int32 sizes, znear default
    0.2), filled through one numpy buffer (the struct is 19 packed 4-byte
    fields) rather than field by field."""
    n = len(cams)
    buf = np.empty((max(1, n), 19), np.float32)
    if n:
        buf[:n, 0:9] = np.asarray([np.asarray(c.R, np.float32).reshape(9) for c in cams], np.float32)
        buf[:n, 9:12] = np.asarray([np.asarray(c.pos, np.float32).reshape(3) for c in cams], np.float32)
        buf[:n, 12:16] = np.asarray([(c.fx, c.fy, c.cx, c.cy) for c in cams], np.float64).astype(np.float32)
        buf[:n, 18] = np.asarray([getattr(c, "near", 0.2) for c in cams], np.float64).astype(np.float32)
        buf[:n].view(np.int32)[:, 16:18] = np.asarray([(int(c.width), int(c.height)) for c in cams], np.int32)
    assert ctypes.sizeof(vy_camera) == 19 * 4
    return (vy_camera * max(1, n)).from_buffer_copy(buf)


def _dev(a, dtype, device):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dtype)


class Scene:
    """Device copy of a hierarchy (scenegen.Scene or any object with the same
    arrays) plus the library's packed workspace (vy_scene_upload)."""

    def __init__(self, host_scene, device="cuda", stream=None):
        import torch
        L = lib()
        self.n = int(host_scene.parent.shape[0])
        self.host = host_scene
        i32, f32 = torch.int32, torch.float32
        self.arrays = dict(
            parent=_dev(host_scene.parent, i32, device), first_child=_dev(host_scene.first_child, i32, device),
            child_count=_dev(host_scene.child_count, i32, device),
            aabb_lo=_dev(host_scene.aabb_lo, f32, device), aabb_hi=_dev(host_scene.aabb_hi, f32, device),
            mean=_dev(host_scene.mean, f32, device), log_scale=_dev(host_scene.log_scale, f32, device),
            quat=_dev(host_scene.quat, f32, device), opacity_logit=_dev(host_scene.opacity_logit, f32, device),
            sh=_dev(host_scene.sh.reshape(self.n, 48), f32, device))
        d = vy_scene_desc()
        d.n_nodes = self.n
        for k, t in self.arrays.items():
            setattr(d, k, t.data_ptr())
        nb = L.vy_scene_workspace_bytes(self.n)
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        check(L.vy_scene_upload(ctypes.byref(d), ctypes.c_void_p(self.ws.data_ptr()), nb, _stream(stream),
                                ctypes.byref(h)), "vy_scene_upload")
        self.handle = h
        # the packed copy replaces the per-attribute arrays (except sh, which is borrowed)
        torch.cuda.current_stream().synchronize()
        keep = self.arrays["sh"]
        self.arrays = {"sh": keep}

    @classmethod
    def from_tensors(cls, tree: dict, params: dict, stream=None):
        """Upload from device tensors: `tree` holds parent, first_child,
        child_count (int32) and aabb_lo, aabb_hi (float32 [n, 3]); `params`
        holds mean [n, 3], log_scale [n, 3], quat [n, 4], opacity_logit [n] and
        sh [n, 16, 3] (float32, contiguous). The sh tensor is borrowed."""
        import torch
        self = cls.__new__(cls)
        L = lib()
        self.n = int(tree["parent"].shape[0])
        self.host = None
        arrays = dict(tree)
        arrays.update(params)
        d = vy_scene_desc()
        d.n_nodes = self.n
        for k in ("parent", "first_child", "child_count", "aabb_lo", "aabb_hi", "mean", "log_scale", "quat",
                  "opacity_logit", "sh"):
            t = arrays[k]
            if not (t.is_cuda and t.is_contiguous()):
                raise VoyagerError(VY_ERR_ARG, f"{k} must be a contiguous device tensor")
            setattr(d, k, t.data_ptr())
        nb = L.vy_scene_workspace_bytes(self.n)
        self.ws = torch.empty(nb, dtype=torch.uint8, device=arrays["mean"].device)
        h = ctypes.c_void_p()
        check(L.vy_scene_upload(ctypes.byref(d), ctypes.c_void_p(self.ws.data_ptr()), nb, _stream(stream),
                                ctypes.byref(h)), "vy_scene_upload")
        self.handle = h
        self.arrays = {"sh": arrays["sh"]}
        return self

    def update_gaussians(self, params: dict, stream=None):
        """vy_scene_update_gaussians: repack mean [n, 3], log_scale [n, 3],
        quat [n, 4], opacity_logit [n] and sh [n, 16, 3] (contiguous float32
        device tensors; sh is borrowed from now on) over the same tree."""
        for k in ("mean", "log_scale", "quat", "opacity_logit", "sh"):
            t = params[k]
            if not (t.is_cuda and t.is_contiguous()) or t.shape[0] != self.n:
                raise VoyagerError(VY_ERR_ARG, f"{k} must be a contiguous device tensor with {self.n} rows")
        check(lib().vy_scene_update_gaussians(self.handle, *[ctypes.c_void_p(params[k].data_ptr()) for k in
                                                             ("mean", "log_scale", "quat", "opacity_logit", "sh")],
                                              _stream(stream)), "vy_scene_update_gaussians")
        self.arrays = {"sh": params["sh"]}

    def partition(self, device="cuda", stream=None):
        """vy_scene_partition: the subtree partition that VY_CUT_CHUNKED
        searches use (its workspace is kept with the scene)."""
        import torch
        nb = int(lib().vy_scene_partition_bytes(self.n))
        self.part_ws = torch.empty(nb, dtype=torch.uint8, device=device)
        check(lib().vy_scene_partition(self.handle, ctypes.c_void_p(self.part_ws.data_ptr()), nb, _stream(stream)),
              "vy_scene_partition")

    def validate(self, stream=None) -> int:
        nb = ctypes.c_int64()
        check(lib().vy_scene_validate(self.handle, ctypes.byref(nb), _stream(stream)), "vy_scene_validate")
        return int(nb.value)

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().vy_scene_free(self.handle)
                self.handle = None
        except Exception:
            pass


class Cut:
    """A cut handle (frontier + cut ids on the device)."""

    def __init__(self, scene: Scene, device="cuda"):
        import torch
        L = lib()
        self.scene = scene
        nb = L.vy_cut_workspace_bytes(scene.n)
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        check(L.vy_cut_create(scene.handle, ctypes.c_void_p(self.ws.data_ptr()), nb, ctypes.byref(h)),
              "vy_cut_create")
        self.handle = h

    def counts(self, stream=None):
        nf, nc = ctypes.c_int64(), ctypes.c_int64()
        check(lib().vy_cut_counts(self.handle, ctypes.byref(nf), ctypes.byref(nc), _stream(stream)),
              "vy_cut_counts")
        return int(nf.value), int(nc.value)

    def ids(self, stream=None):
        """(frontier, cut) as int64 numpy arrays (synchronises)."""
        import torch
        nf, nc = self.counts(stream)
        pf, pc, pn = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        check(lib().vy_cut_arrays(self.handle, ctypes.byref(pf), ctypes.byref(pc), ctypes.byref(pn)),
              "vy_cut_arrays")
        F = np.empty(nf, np.int32)
        C = np.empty(nc, np.int32)
        if nf:
            _copy_d2h(F, pf.value)
        if nc:
            _copy_d2h(C, pc.value)
        return F.astype(np.int64), C.astype(np.int64)

    def set_frontier(self, ids, stream=None):
        import torch
        t = torch.as_tensor(np.asarray(ids, np.int32), device="cuda")
        check(lib().vy_cut_set_frontier(self.handle, ctypes.c_void_p(t.data_ptr()), int(t.numel()),
                                        _stream(stream)), "vy_cut_set_frontier")
        torch.cuda.current_stream().synchronize()

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().vy_cut_free(self.handle)
                self.handle = None
        except Exception:
            pass


class _DevView:
    """Zero-copy view of library-owned device memory for torch.as_tensor."""

    def __init__(self, ptr: int, shape, typestr: str):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (int(ptr), False),
                                         "version": 2, "strides": None}


def device_view(ptr: int, shape, dtype=np.int32):
    """torch tensor aliasing `ptr` (device memory owned by the library)."""
    import torch
    typestr = np.dtype(dtype).str
    return torch.as_tensor(_DevView(ptr, shape, typestr), device="cuda")


def _copy_d2h(dst: np.ndarray, src_ptr: int):
    import torch
    torch.cuda.current_stream().synchronize()
    dst[...] = device_view(src_ptr, dst.shape, dst.dtype).cpu().numpy()


class RenderContext:
    def __init__(self, max_gaussians, max_width, max_height, max_pairs, device="cuda"):
        import torch
        L = lib()
        nb = L.vy_render_workspace_bytes(int(max_gaussians), int(max_width), int(max_height), int(max_pairs))
        if nb == 0:
            raise VoyagerError(VY_ERR_ARG, "vy_render_workspace_bytes: invalid sizes")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        check(L.vy_render_ctx_create(int(max_gaussians), int(max_width), int(max_height), int(max_pairs),
                                     ctypes.c_void_p(self.ws.data_ptr()), nb, ctypes.byref(h)),
              "vy_render_ctx_create")
        self.handle = h
        self.max_width, self.max_height, self.max_pairs = int(max_width), int(max_height), int(max_pairs)

    def status(self, stream=None):
        n_pairs, n_vis = ctypes.c_int64(), ctypes.c_int64()
        rc = lib().vy_render_status(self.handle, ctypes.byref(n_pairs), ctypes.byref(n_vis), _stream(stream))
        return rc, int(n_pairs.value), int(n_vis.value)

    def saved(self, width, height, evals=False, last=False):
        """(T_final, n_contrib[, n_eval][, last contributor]) of the last frame
        rendered with save_state (synchronises)."""
        pt, pn, pe, pl, pm = (ctypes.c_void_p() for _ in range(5))
        check(lib().vy_render_saved(self.handle, ctypes.byref(pt), ctypes.byref(pn), ctypes.byref(pe),
                                    ctypes.byref(pl), ctypes.byref(pm)), "vy_render_saved")
        T = np.empty((height, width), np.float32)
        N = np.empty((height, width), np.int32)
        _copy_d2h(T, pt.value)
        _copy_d2h(N, pn.value)
        out = [T, N]
        if evals:
            E = np.empty((height, width), np.int32)
            _copy_d2h(E, pe.value)
            out.append(E)
        if last:
            Lc = np.empty((height, width), np.int32)
            _copy_d2h(Lc, pl.value)
            out.append(Lc)
        return tuple(out)

    def pairs(self, width, height, raw=False):
        """Last frame's sorted pairs (tile ids, cut positions) and tile ranges
        (synchronises). The device keys hold the tile id in their low 16 bits
        and the pair's pixel box within the tile above it; `raw` returns them
        whole, else the tile ids."""
        rc, n_pairs, n_vis = self.status()
        check(rc, "vy_render_status")
        pk, pv, pr = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        check(lib().vy_render_pairs(self.handle, ctypes.byref(pk), ctypes.byref(pv), ctypes.byref(pr)),
              "vy_render_pairs")
        ntiles = ((width + 15) // 16) * ((height + 15) // 16)
        keys = np.empty(n_pairs, np.uint32)
        vals = np.empty(n_pairs, np.uint32)
        ranges = np.empty((ntiles, 2), np.uint32)
        if n_pairs:
            _copy_d2h(keys, pk.value)
            _copy_d2h(vals, pv.value)
        _copy_d2h(ranges, pr.value)
        return (keys if raw else keys & np.uint32(0xFFFF)), vals, ranges

    def projected(self, n):
        """Projected records of the first n cut positions (synchronises): rec0, rec1,
        rec2 as float32 [n, 4] and the binning record as uint32 [n, 4] (tile rect
        corners, kept-tile mask, pair count)."""
        ptrs = [ctypes.c_void_p() for _ in range(4)]
        check(lib().vy_render_projected(self.handle, *[ctypes.byref(p) for p in ptrs]), "vy_render_projected")
        out = []
        for p, dt in zip(ptrs, (np.float32, np.float32, np.float32, np.uint32)):
            a = np.empty((n, 4), dt)
            if n:
                _copy_d2h(a, p.value)
            out.append(a)
        return out

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().vy_render_ctx_free(self.handle)
                self.handle = None
        except Exception:
            pass


# ----------------------------------------------------------------------------
# C-ABI-named entry points
# ----------------------------------------------------------------------------

def vy_scene_upload(host_scene, device="cuda", stream=None) -> Scene:
    return Scene(host_scene, device, stream)


def vy_lod_cut(scene: Scene, cam, tau: float, prev: Cut | None = None, out: Cut | None = None,
               mode: int = VY_CUT_FRONTIER, stream=None) -> Cut:
    """Enqueue the LoD cut; returns `out` (a new Cut when None)."""
    if out is None:
        out = Cut(scene)
    c = make_camera(cam)
    check(lib().vy_lod_cut(scene.handle, ctypes.byref(c), float(tau), prev.handle if prev is not None else None,
                           out.handle, int(mode), _stream(stream)), "vy_lod_cut")
    return out


def vy_render(scene: Scene, cut: Cut, cam, ctx: RenderContext, image=None, alpha_filter=False,
              bg=(0.0, 0.0, 0.0), save_state=False, split_min_pairs=0, walk=0, lut_entries=0, band_jobs=0,
              stream=None):
    """Enqueue rendering of `cut` into `image` (torch float32 [3, H, W] on the device)."""
    import torch
    if image is None:
        image = torch.empty((3, int(cam.height), int(cam.width)), dtype=torch.float32, device="cuda")
    if image.dtype != torch.float32 or not image.is_contiguous() or tuple(image.shape) != (3, cam.height, cam.width):
        raise VoyagerError(VY_ERR_ARG, "image must be a contiguous float32 tensor of shape (3, H, W)")
    o = _render_opts(alpha_filter, bg, save_state, split_min_pairs, walk, lut_entries, band_jobs)
    c = make_camera(cam)
    check(lib().vy_render(scene.handle, cut.handle, ctypes.byref(c), ctypes.byref(o),
                          ctypes.c_void_p(image.data_ptr()), ctx.handle, _stream(stream)), "vy_render")
    return image


BATCH_MAX_VIEWS, BATCH_MAX_TILES = 64, 65536


class BatchContext:
    """Buffers shared by the frames of a batch (vy_batch_ctx): at most
    max_views views, max_gaussians cut Gaussians and max_tiles tiles in all,
    max_pairs pairs."""

    def __init__(self, max_views, max_gaussians, max_tiles, max_pairs, device="cuda"):
        import torch
        L = lib()
        nb = int(L.vy_batch_workspace_bytes(int(max_views), int(max_gaussians), int(max_tiles), int(max_pairs)))
        if nb == 0:
            raise VoyagerError(VY_ERR_ARG, "BatchContext: invalid capacities")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        check(L.vy_batch_ctx_create(int(max_views), int(max_gaussians), int(max_tiles), int(max_pairs),
                                    ctypes.c_void_p(self.ws.data_ptr()), nb, ctypes.byref(h)), "vy_batch_ctx_create")
        self.handle = h
        self.max_views = int(max_views)

    def status(self, stream=None):
        npairs, nvis = ctypes.c_int64(), ctypes.c_int64()
        rc = lib().vy_batch_status(self.handle, ctypes.byref(npairs), ctypes.byref(nvis), _stream(stream))
        return rc, int(npairs.value), int(nvis.value)

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().vy_batch_ctx_free(self.handle)
                self.handle = None
        except Exception:
            pass


def vy_render_batch(views, ctx: BatchContext, alpha_filter=False, bg=(0.0, 0.0, 0.0), walk=0, lut_entries=0,
                    band_jobs=0, stream=None):
    """Enqueue one batched render of `views`: (scene, cut, cam, image) tuples,
    image a contiguous float32 [3, H, W] device tensor. Returns the images."""
    import torch
    n = len(views)
    arr = (vy_view * max(1, n))()
    for i, (scene, cut, cam, image) in enumerate(views):
        if image.dtype != torch.float32 or not image.is_contiguous() or \
                tuple(image.shape) != (3, cam.height, cam.width):
            raise VoyagerError(VY_ERR_ARG, "image must be a contiguous float32 tensor of shape (3, H, W)")
        arr[i].scene = scene.handle.value if isinstance(scene.handle, ctypes.c_void_p) else scene.handle
        arr[i].cut = cut.handle.value if isinstance(cut.handle, ctypes.c_void_p) else cut.handle
        arr[i].cam = make_camera(cam)
        arr[i].image = image.data_ptr()
    o = _render_opts(alpha_filter, bg, False, 0, walk, lut_entries, band_jobs)
    check(lib().vy_render_batch(arr, n, ctypes.byref(o), ctx.handle, _stream(stream)), "vy_render_batch")
    return [v[3] for v in views]


def partition_plan(parent, first_child, child_count):
    """vy_partition_plan on host arrays: dict of sub_of, local, sub_root,
    sub_rec and chunk_sub (numpy int32)."""
    parent = np.ascontiguousarray(parent, np.int32)
    first_child = np.ascontiguousarray(first_child, np.int32)
    child_count = np.ascontiguousarray(child_count, np.int32)
    n = len(parent)
    out = {k: np.empty(n + (1 if k in ("sub_rec", "chunk_sub") else 0), np.int32)
           for k in ("sub_of", "local", "sub_root", "sub_rec", "chunk_sub")}
    ns, nc = ctypes.c_int64(), ctypes.c_int64()
    ptr = lambda a: ctypes.c_void_p(a.ctypes.data)   # noqa: E731
    check(lib().vy_partition_plan(n, ptr(parent), ptr(first_child), ptr(child_count), ptr(out["sub_of"]),
                                  ptr(out["local"]), ctypes.byref(ns), ptr(out["sub_root"]), ptr(out["sub_rec"]),
                                  ptr(out["chunk_sub"]), ctypes.byref(nc)), "vy_partition_plan")
    out["sub_root"] = out["sub_root"][:ns.value]
    out["sub_rec"] = out["sub_rec"][:ns.value + 1]
    out["chunk_sub"] = out["chunk_sub"][:nc.value + 1]
    return out


# capacities of vy_render_noalloc's static scratch (vy.h)
NOALLOC_SCRATCH_BYTES = 64 << 20
NOALLOC_MAX_GAUSSIANS = 1 << 18
NOALLOC_MAX_PAIRS = 1 << 20
NOALLOC_MAX_WIDTH, NOALLOC_MAX_HEIGHT = 1280, 720


def vy_render_noalloc(scene: Scene, cut: Cut, cam, image=None, counts=None, alpha_filter=False,
                      bg=(0.0, 0.0, 0.0), walk=0, lut_entries=0, band_jobs=0, stream=None):
    """Enqueue rendering of `cut` into `image` with the library's static
    scratch instead of a context (no allocation inside the call). `counts`: a
    device int32/uint32 tensor of 4 elements receiving {pairs needed,
    Gaussians with pairs, cut size if over capacity else 0, device errors},
    or None. Returns `image`."""
    import torch
    if image is None:
        image = torch.empty((3, int(cam.height), int(cam.width)), dtype=torch.float32, device="cuda")
    if image.dtype != torch.float32 or not image.is_contiguous() or tuple(image.shape) != (3, cam.height, cam.width):
        raise VoyagerError(VY_ERR_ARG, "image must be a contiguous float32 tensor of shape (3, H, W)")
    if counts is not None and (counts.numel() < 4 or counts.element_size() != 4 or not counts.is_contiguous()):
        raise VoyagerError(VY_ERR_ARG, "counts must be a contiguous 32-bit tensor of at least 4 elements")
    o = _render_opts(alpha_filter, bg, False, 0, walk, lut_entries, band_jobs)
    c = make_camera(cam)
    check(lib().vy_render_noalloc(scene.handle, cut.handle, ctypes.byref(c), ctypes.byref(o),
                                  ctypes.c_void_p(image.data_ptr()),
                                  ctypes.c_void_p(counts.data_ptr()) if counts is not None else None,
                                  _stream(stream)), "vy_render_noalloc")
    return image


def measure_peaks(stream=None):
    """The device's practical FP32 FMA rate (TFLOP/s) and v_exp_f32 rate
    (G/s), from the library's probe kernels (synchronises)."""
    import torch
    L = lib()
    nb = int(L.vy_measure_peaks_bytes())
    buf = torch.empty(nb // 4, dtype=torch.float32, device="cuda")
    f, e = ctypes.c_double(), ctypes.c_double()
    check(L.vy_measure_peaks(ctypes.c_void_p(buf.data_ptr()), nb, ctypes.byref(f), ctypes.byref(e), _stream(stream)),
          "vy_measure_peaks")
    return dict(fma_fp32_tflops=f.value, exp_f32_gops=e.value)


def _render_opts(alpha_filter=False, bg=(0.0, 0.0, 0.0), save_state=False, split_min_pairs=0, walk=0, lut_entries=0,
                 band_jobs=0):
    o = vy_render_opts()
    o.alpha_filter = 1 if alpha_filter else 0
    for i in range(3):
        o.bg[i] = float(bg[i])
    o.save_state = 1 if save_state else 0
    o.split_min_pairs = int(split_min_pairs)
    o.walk = int(walk)
    o.lut_entries = int(lut_entries)
    o.band_jobs = int(band_jobs)
    return o


def vy_walkthrough(scene: Scene, cams, tau: float, cuts, ctxs, images, streams=None, prev: Cut | None = None,
                   mode: int = VY_CUT_FRONTIER, alpha_filter=False, bg=(0.0, 0.0, 0.0), walk=0, lut_entries=0,
                   band_jobs=0, stats=None, frame_ms=False, stream=None):
    """Enqueue the frames of a camera path with len(cuts) frames in flight.
    Frame i searches its cut from frame i-1's (from `prev` for frame 0, a full
    search when None) into cuts[i % depth] and renders it with ctxs[i % depth]
    on streams[i % depth] (torch streams; default: the current stream, depth
    1) into images[i % len(images)] (torch float32 [3, H, W]; len(images) a
    multiple of depth). `stats`: a device tensor of at least 32 bytes per frame
    for the per-frame records (decode with serving.STATS_DTYPE), or None.
    Returns the per-frame GPU milliseconds (numpy, after synchronising) when
    `frame_ms`, else None."""
    import torch
    depth = len(cuts)
    if streams is None:
        if depth != 1:
            raise VoyagerError(VY_ERR_ARG, "vy_walkthrough: give one stream per slot when depth > 1")
        streams = [torch.cuda.current_stream()]
    if len(ctxs) != depth or len(streams) != depth:
        raise VoyagerError(VY_ERR_ARG, "vy_walkthrough: cuts, ctxs and streams must have the same length")
    n = len(cams)
    for im in images:
        if im.dtype != torch.float32 or not im.is_contiguous() or im.dim() != 3 or im.shape[0] != 3:
            raise VoyagerError(VY_ERR_ARG, "images must be contiguous float32 tensors of shape (3, H, W)")
    shapes = [(int(im.shape[1]), int(im.shape[2])) for im in images]
    for i, cam in enumerate(cams):
        if shapes[i % len(images)] != (cam.height, cam.width):
            raise VoyagerError(VY_ERR_ARG, f"frame {i}: image shape differs from the camera's size")
    if stats is not None and stats.numel() * stats.element_size() < 32 * n:
        raise VoyagerError(VY_ERR_ARG, "stats needs 32 bytes per frame")
    cam_arr = make_cameras(cams)
    o = _render_opts(alpha_filter, bg, False, 0, walk, lut_entries, band_jobs)
    P = ctypes.c_void_p
    cut_arr = (P * depth)(*[c.handle for c in cuts])
    ctx_arr = (P * depth)(*[c.handle for c in ctxs])
    st_arr = (P * depth)(*[s.cuda_stream for s in streams])
    img_arr = (P * max(1, len(images)))(*[im.data_ptr() for im in images])
    ms = (ctypes.c_float * max(1, n))() if frame_ms else None
    check(lib().vy_walkthrough(scene.handle, cam_arr, n, float(tau), int(mode), ctypes.byref(o),
                               prev.handle if prev is not None else None, depth, cut_arr, ctx_arr, st_arr, img_arr,
                               len(images), P(stats.data_ptr()) if stats is not None else None, ms, _stream(stream)),
          "vy_walkthrough")
    return np.frombuffer(bytes(ms), dtype=np.float32)[:n].copy() if frame_ms else None


def vy_render_backward(scene: Scene, cut: Cut, cam, ctx: RenderContext, dL_dimage, quat_raw=None,
                       mean2d=False, stream=None):
    """Gradients of the last vy_render(..., save_state=True) on `ctx` for
    dL/dimage (torch float32 [3, H, W] on the device). Returns a dict of
    node-indexed torch tensors: mean [n, 3], log_scale [n, 3], quat [n, 4]
    (for `quat_raw`, the quaternions as uploaded, when given; else for the unit
    quaternion), opacity_logit [n], sh [n, 16, 3] (and mean2d [n, 2])."""
    import torch
    n = scene.n
    if dL_dimage.dtype != torch.float32 or not dL_dimage.is_contiguous() or \
            tuple(dL_dimage.shape) != (3, cam.height, cam.width):
        raise VoyagerError(VY_ERR_ARG, "dL_dimage must be a contiguous float32 tensor of shape (3, H, W)")
    dev = dL_dimage.device
    out = dict(mean=torch.zeros((n, 3), device=dev), log_scale=torch.zeros((n, 3), device=dev),
               quat=torch.zeros((n, 4), device=dev), opacity_logit=torch.zeros(n, device=dev),
               sh=torch.zeros((n, 16, 3), device=dev))
    if mean2d:
        out["mean2d"] = torch.zeros((n, 2), device=dev)
    g = vy_grads()
    for k, t in out.items():
        setattr(g, k, t.data_ptr())
    g.quat_raw = quat_raw.data_ptr() if quat_raw is not None else None
    c = make_camera(cam)
    check(lib().vy_render_backward(scene.handle, cut.handle, ctypes.byref(c), ctypes.c_void_p(dL_dimage.data_ptr()),
                                   ctypes.byref(g), ctx.handle, _stream(stream)), "vy_render_backward")
    return out


def profile_begin(capacity=1 << 16):
    check(lib().vy_profile_begin(int(capacity)), "vy_profile_begin")


def profile_end():
    ms = (ctypes.c_double * len(STAGES))()
    n = (ctypes.c_int64 * len(STAGES))()
    check(lib().vy_profile_end(ms, n), "vy_profile_end")
    return {STAGES[i]: (float(ms[i]), int(n[i])) for i in range(len(STAGES))}
