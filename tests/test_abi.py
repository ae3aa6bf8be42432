"""CPU-only checks of the C-ABI library: it loads, exports every entry point
declared in include/*.h, sizes workspaces, and rejects bad arguments before
touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(os.path.join(ROOT, "include", h) for h in os.listdir(os.path.join(ROOT, "include"))
                 if h.endswith(".h"))


def _header_text():
    return "\n".join(open(h).read() for h in HEADERS)


def _lib():
    vy = pytest.importorskip("paper_2506_02774_amd")
    try:
        return vy, vy.lib()
    except ImportError as e:
        pytest.fail(f"library not built: {e}")


def declared_functions():
    src = re.sub(r"/\*.*?\*/", "", _header_text(), flags=re.S)
    return sorted(set(re.findall(r"\b(vy_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    vy, L = _lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    # and nm agrees (the symbols are real exports, not ctypes lookups of something else)
    out = os.popen(f"nm -D --defined-only {vy.LIB_PATH}").read()
    for n in names:
        assert re.search(rf"\bT {n}\b", out), n


def test_workspace_queries():
    vy, L = _lib()
    assert L.vy_scene_workspace_bytes(0) == 0
    assert L.vy_scene_workspace_bytes(1000) >= 1000 * 84
    assert L.vy_cut_workspace_bytes(1000) >= 1000 * 16
    a = L.vy_render_workspace_bytes(1000, 64, 64, 10_000)
    b = L.vy_render_workspace_bytes(1000, 64, 64, 20_000)
    assert b - a >= 10_000 * 16
    assert L.vy_render_workspace_bytes(0, 64, 64, 10) == 0


def test_argument_errors_without_gpu():
    vy, L = _lib()
    h = ctypes.c_void_p()
    assert L.vy_scene_upload(None, None, 0, None, ctypes.byref(h)) == vy.VY_ERR_ARG
    assert b"NULL" in L.vy_last_error()
    d = vy.vy_scene_desc()
    d.n_nodes = 0
    assert L.vy_scene_upload(ctypes.byref(d), ctypes.c_void_p(1), 1 << 20, None, ctypes.byref(h)) == vy.VY_ERR_ARG
    assert L.vy_lod_cut(None, None, 1.0, None, None, 0, None) == vy.VY_ERR_ARG
    assert L.vy_render(None, None, None, None, None, None, None) == vy.VY_ERR_ARG
    assert L.vy_render_ctx_create(10, 64, 64, 100, None, 0, ctypes.byref(h)) == vy.VY_ERR_ARG
    assert L.vy_profile_begin(0) == vy.VY_ERR_ARG
    f, e = ctypes.c_double(), ctypes.c_double()
    nb = L.vy_measure_peaks_bytes()
    assert nb >= 4 * 256
    assert L.vy_measure_peaks(None, nb, ctypes.byref(f), ctypes.byref(e), None) == vy.VY_ERR_ARG
    assert L.vy_measure_peaks(ctypes.c_void_p(1), nb - 1, ctypes.byref(f), ctypes.byref(e), None) == vy.VY_ERR_ARG
    assert L.vy_stage_name(13) == b"blend" and L.vy_stage_name(12) == b"blend_plan" and L.vy_stage_name(99) == b"?"


def declared_arity():
    """Parameter count of every function declared in include/*.h."""
    src = re.sub(r"/\*.*?\*/", "", _header_text(), flags=re.S)
    out = {}
    for name, params in re.findall(r"\b(vy_[a-z0-9_]+)\s*\(([^()]*)\)\s*;", src):
        p = params.strip()
        out[name] = 0 if p in ("", "void") else p.count(",") + 1
    return out


def test_binding_matches_header_arity():
    """The ctypes signatures of the binding take exactly the parameters that the
    header declares (a mismatch would only show up as a failed call on a GPU)."""
    vy, L = _lib()
    decl = declared_arity()
    assert len(decl) >= 20
    for name, n in decl.items():
        f = getattr(L, name)
        assert f.argtypes is not None, name
        assert len(f.argtypes) == n, (name, len(f.argtypes), n)


def test_noalloc_limits_match_the_header():
    vy, L = _lib()
    text = _header_text()
    want = dict(VY_NOALLOC_SCRATCH_BYTES=vy.NOALLOC_SCRATCH_BYTES, VY_NOALLOC_MAX_GAUSSIANS=vy.NOALLOC_MAX_GAUSSIANS,
                VY_NOALLOC_MAX_PAIRS=vy.NOALLOC_MAX_PAIRS, VY_NOALLOC_MAX_WIDTH=vy.NOALLOC_MAX_WIDTH,
                VY_NOALLOC_MAX_HEIGHT=vy.NOALLOC_MAX_HEIGHT)
    for name, v in want.items():
        m = re.search(rf"#define {name} \(?([0-9]+)u? *(<< *([0-9]+))?\)?", text)
        assert m, name
        got = int(m.group(1)) << (int(m.group(3)) if m.group(3) else 0)
        assert got == v, name
    # the fixed layout fits the static array. vy_render_workspace_bytes counts the
    # split-tile buffers (which the static layout leaves out and whose size does
    # not depend on the arguments); the rest of a 1-Gaussian 16x16 context is
    # more than 4096 bytes, so need - split_extra bounds the layout from above
    need = L.vy_render_workspace_bytes(vy.NOALLOC_MAX_GAUSSIANS, vy.NOALLOC_MAX_WIDTH, vy.NOALLOC_MAX_HEIGHT,
                                       vy.NOALLOC_MAX_PAIRS)
    split_extra = L.vy_render_workspace_bytes(1, 16, 16, 1) - 4096
    assert need - split_extra <= vy.NOALLOC_SCRATCH_BYTES


def test_noalloc_rejects_before_touching_the_gpu():
    vy, L = _lib()
    c = vy.vy_camera()
    c.width, c.height, c.fx, c.fy, c.znear = vy.NOALLOC_MAX_WIDTH + 1, 64, 100.0, 100.0, 0.2
    img = ctypes.c_void_p(1 << 40)       # never dereferenced: the size check comes first
    assert L.vy_render_noalloc(None, None, ctypes.byref(c), None, img, None, None) == vy.VY_ERR_ARG
    assert b"static scratch" in L.vy_last_error()
    c.width = 64
    o = vy.vy_render_opts()
    o.save_state = 1
    assert L.vy_render_noalloc(None, None, ctypes.byref(c), ctypes.byref(o), img, None, None) == vy.VY_ERR_ARG
    assert L.vy_render_noalloc(None, None, None, None, img, None, None) == vy.VY_ERR_ARG


def test_camera_array_matches_single_cameras():
    """make_cameras (one numpy buffer for a whole camera path) gives the same
    vy_camera bytes as make_camera per camera: float32 rounding of the
    intrinsics, int32 sizes, the default near plane, any camera-like object."""
    import numpy as np
    import scenegen
    import paper_2506_02774_amd as vy

    class Cam:
        pass

    c = Cam()
    c.R, c.pos = np.eye(3) * 0.5, [1.0, -2.0, 3.25]
    c.fx, c.fy, c.cx, c.cy, c.width, c.height = 100.123456789, 99.5, 32.25, 16, 64, 48
    cams = list(scenegen.walkthrough(scenegen.CONFIGS["tiny"])) + [
        scenegen.identity_camera(64, 48), scenegen.look_camera([0.0, 0.0, 50.0], 0.3, -0.2, 100, 37), c]
    one = (vy.vy_camera * len(cams))(*[vy.make_camera(x) for x in cams])
    assert bytes(vy.make_cameras(cams)) == bytes(one)
    assert len(bytes(vy.make_cameras([]))) == ctypes.sizeof(vy.vy_camera)
