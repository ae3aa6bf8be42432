"""CPU checks of the serving runtime's host logic (vy_serve.h): the device
memory arena against a plain first-fit model, the admission and scheduling
policy through vy_server_simulate (the same policy code as vy_server_run,
driven by a model of the GPU), and the C struct layouts of the binding."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _vy():
    vy = pytest.importorskip("paper_2506_02774_amd")
    try:
        vy.lib()
    except ImportError as e:
        pytest.fail(f"library not built: {e}")
    from paper_2506_02774_amd import serving
    return vy, serving


FAKE_BASE = 1 << 40          # never dereferenced: the arena only does bookkeeping


# ------------------------------------------------------------------ arena ----

class FirstFit:
    """Plain model: a sorted list of free (offset, size), 256-byte granules."""

    def __init__(self, nbytes):
        self.size = nbytes // 256 * 256
        self.free = [(0, self.size)]
        self.live = {}

    def alloc(self, n):
        need = -(-n // 256) * 256
        for i, (o, s) in enumerate(self.free):
            if s >= need:
                if s == need:
                    self.free.pop(i)
                else:
                    self.free[i] = (o + need, s - need)
                self.live[o] = need
                return o
        return None

    def release(self, o):
        s = self.live.pop(o)
        self.free.append((o, s))
        self.free.sort()
        merged = []
        for fo, fs in self.free:
            if merged and merged[-1][0] + merged[-1][1] == fo:
                merged[-1] = (merged[-1][0], merged[-1][1] + fs)
            else:
                merged.append((fo, fs))
        self.free = merged


def test_arena_matches_first_fit_model():
    vy, serving = _vy()
    rng = np.random.default_rng(5)
    total = 1 << 24
    a = serving.Arena(total, base=FAKE_BASE)
    m = FirstFit(total)
    live = []
    for step in range(3000):
        if live and (rng.random() < 0.45 or len(live) > 40):
            k = int(rng.integers(len(live)))
            off = live.pop(k)
            a.release(FAKE_BASE + off)
            m.release(off)
        else:
            n = int(rng.integers(1, 1 << 20))
            want = m.alloc(n)
            if want is None:
                with pytest.raises(vy.VoyagerError) as e:
                    a.alloc(n)
                assert e.value.code == vy.VY_ERR_CAPACITY
            else:
                got = a.alloc(n) - FAKE_BASE
                assert got == want, step
                assert got % 256 == 0
                live.append(got)
        st = a.stats()
        assert st["used"] == sum(m.live.values())
        assert st["n_live"] == len(m.live)
        assert st["n_free_blocks"] == len(m.free)
        assert st["largest_free"] == max([s for _, s in m.free], default=0)
    # blocks never overlap
    spans = sorted((o, o + s) for o, s in m.live.items())
    assert all(b0 <= a0 for (_, b0), (a0, _) in zip(spans, spans[1:]))
    for off in live:
        a.release(FAKE_BASE + off)
    assert a.stats() == dict(used=0, largest_free=total, n_live=0, n_free_blocks=1)


def test_arena_errors():
    vy, serving = _vy()
    with pytest.raises(vy.VoyagerError):
        serving.Arena(1 << 20, base=FAKE_BASE + 8)          # misaligned
    a = serving.Arena(1 << 20, base=FAKE_BASE)
    with pytest.raises(vy.VoyagerError) as e:
        a.alloc((1 << 20) + 1)
    assert e.value.code == vy.VY_ERR_CAPACITY
    p = a.alloc(1000)
    with pytest.raises(vy.VoyagerError) as e:
        a.release(p + 256)                                   # not the start of a block
    assert e.value.code == vy.VY_ERR_ARG
    a.release(p)
    with pytest.raises(vy.VoyagerError):
        a.release(p)                                         # twice
    with pytest.raises(vy.VoyagerError):
        a.alloc(0)


# ----------------------------------------------------------------- policy ----

def _trace(serving, items):
    """items: (session, t_arrival) in arrival order -> request array."""
    return serving.build_requests((s, t, None, 0) for s, t in items)


def test_simulated_serial_stream_is_fifo():
    vy, serving = _vy()
    a = serving.Arena(1 << 20, base=FAKE_BASE)
    reqs, n = _trace(serving, [(0, 0.0), (1, 0.0), (0, 0.0), (1, 0.0), (2, 0.5)])
    res, cnt = serving.simulate(a, 1, 1, 8, [1000, 1000, 1000], reqs, n, [1.0, 2.0, 1.0, 2.0, 1.0])
    # one stream, one frame at a time, oldest request first: back to back
    assert res["t_start"].tolist() == [0.0, 1.0, 3.0, 4.0, 6.0]
    assert res["t_done"].tolist() == [1.0, 3.0, 4.0, 6.0, 7.0]
    assert res["stream"].tolist() == [0] * 5 and not res["status"].any()
    assert cnt["admitted"] == 3 and cnt["waited"] == 0 and cnt["peak_resident"] == 3
    assert a.stats()["n_live"] == 0                        # every session released


def test_simulated_admission_respects_budget_and_order():
    vy, serving = _vy()
    budget = 3 * (1 << 20)
    a = serving.Arena(budget, base=FAKE_BASE)
    rng = np.random.default_rng(11)
    n_sess, items = 12, []
    sizes = [int(rng.integers(1 << 19, 2 << 20)) for _ in range(n_sess)]
    t = 0.0
    per = {s: int(rng.integers(2, 6)) for s in range(n_sess)}
    left = dict(per)
    while any(left.values()):
        s = int(rng.choice([k for k, v in left.items() if v]))
        items.append((s, t))
        left[s] -= 1
        t += float(rng.exponential(0.05))
    reqs, n = _trace(serving, items)
    service = rng.uniform(0.01, 0.1, n)
    for streams, inflight in [(1, 1), (2, 2), (4, 3)]:
        res, cnt = serving.simulate(a, streams, inflight, 3, sizes, reqs, n, service)
        sess = np.array([s for s, _ in items])
        arr = np.array([t for _, t in items])
        assert not res["status"].any()
        assert np.all(res["t_start"] >= arr - 1e-12) and np.all(res["t_done"] >= res["t_start"])
        assert np.all(res["t_dispatch"] >= res["t_admit"])
        for s in range(n_sess):
            idx = np.flatnonzero(sess == s)
            # a session's frames run in order, each after the previous one ended
            assert np.all(np.diff(res["t_start"][idx]) >= 0)
            assert np.all(res["t_start"][idx][1:] >= res["t_done"][idx][:-1] - 1e-12)
            assert np.all(res["t_admit"][idx] == res["t_admit"][idx][0])
        # never more than 3 resident, never above the budget; all released at the end
        assert cnt["peak_resident"] <= 3 and cnt["peak_bytes"] <= budget
        assert cnt["admitted"] == n_sess and cnt["waited"] > 0
        assert a.stats()["n_live"] == 0
        # residency intervals: at every admission, the resident sessions fit the budget and the slots
        first = {s: int(np.flatnonzero(sess == s)[0]) for s in range(n_sess)}
        last = {s: int(np.flatnonzero(sess == s)[-1]) for s in range(n_sess)}
        spans = [(res["t_admit"][first[s]], res["t_done"][last[s]], s) for s in range(n_sess)]
        for t0, _, s in spans:
            live = [q for (a0, a1, q) in spans if a0 <= t0 < a1]
            assert len(live) <= 3
            assert sum(-(-sizes[q] // 256) * 256 for q in live) <= budget
        # first come, first served: admission order follows first arrivals
        order = sorted(range(n_sess), key=lambda s: (res["t_admit"][first[s]], first[s]))
        assert order == sorted(range(n_sess), key=lambda s: first[s])


def test_simulated_streams_overlap_sessions():
    vy, serving = _vy()
    a = serving.Arena(1 << 24, base=FAKE_BASE)
    items = [(s, 0.0) for _ in range(3) for s in range(4)]
    reqs, n = _trace(serving, items)
    res1, _ = serving.simulate(a, 1, 2, 8, [4096] * 4, reqs, n, [1.0] * n, realtime=False)
    res4, _ = serving.simulate(a, 4, 2, 8, [4096] * 4, reqs, n, [1.0] * n, realtime=False)
    assert res1["t_done"].max() == 12.0
    assert res4["t_done"].max() == 3.0                     # one session per stream
    for s in range(4):
        assert len(set(res4["stream"][s::4].tolist())) == 1    # sessions keep their stream


def test_simulated_growth_rerenders_overflowed_frames():
    vy, serving = _vy()
    a = serving.Arena(1 << 20, base=FAKE_BASE)
    items = [(0, 0.0), (1, 0.0), (0, 0.1), (1, 0.1), (0, 0.2), (1, 0.2), (1, 0.3)]
    need = [50, 50, 50, 250, 50, 50, 600]
    reqs, n = _trace(serving, items)
    res, cnt = serving.simulate(a, 1, 1, 4, [4096, 4096], reqs, n, [0.01] * n, pair_capacity=[100, 100],
                                need_pairs=need)
    # session 1 overflows twice: 100 -> max(2 * 100, 1.25 * 250) = 312 pairs, then -> max(624, 750) = 750
    assert cnt["regrown"] == 2 and cnt["redone"] == 2
    assert cnt["peak_bytes"] >= 4096 + 750 * 16
    assert not res["status"].any() and a.stats()["n_live"] == 0
    # a re-rendered frame starts after its session's earlier frames and ends last of its session
    assert res["t_done"][3] >= res["t_done"][1] and res["t_done"][6] == res["t_done"][[1, 3, 5, 6]].max()
    # capacities the caller fixed (no growth model) only run once
    res2, cnt2 = serving.simulate(a, 1, 1, 4, [4096, 4096], reqs, n, [0.01] * n, pair_capacity=[100, 100])
    assert cnt2["regrown"] == 0 and cnt2["redone"] == 0


def test_simulated_growth_beyond_the_arena_gives_up():
    vy, serving = _vy()
    a = serving.Arena(8192, base=FAKE_BASE)
    reqs, n = _trace(serving, [(0, 0.0), (0, 0.1)])
    res, cnt = serving.simulate(a, 1, 1, 1, [4096], reqs, n, [0.01] * n, pair_capacity=[64], need_pairs=[10, 10**6])
    assert cnt["regrown"] == 0 and cnt["redone"] == 1       # tried, could never fit: the frame stays as it was
    assert a.stats()["n_live"] == 0


def test_simulated_growth_reuses_the_sessions_own_block():
    """A lone session whose larger render block fits only once its own old
    block is given back still grows (8192-byte arena, 4096 fixed, 64 -> 250
    pairs: 4096 + 4000 bytes)."""
    vy, serving = _vy()
    a = serving.Arena(8192, base=FAKE_BASE)
    reqs, n = _trace(serving, [(0, 0.0), (0, 0.1), (0, 0.2)])
    res, cnt = serving.simulate(a, 1, 1, 1, [4096], reqs, n, [0.01] * n, pair_capacity=[64],
                                need_pairs=[100, 200, 10])
    assert cnt["regrown"] == 2 and cnt["redone"] == 2
    assert not res["status"].any() and a.stats()["n_live"] == 0


def test_simulated_growth_when_every_session_waits_for_memory():
    """Two sessions overflow one after the other and neither larger block fits
    beside the other session's memory: one of them keeps its frame as it was
    (flagged) and runs on, and the other grows once it has left."""
    vy, serving = _vy()
    a = serving.Arena(16384, base=FAKE_BASE)
    reqs, n = _trace(serving, [(0, 0.0), (1, 0.0), (0, 0.1), (1, 0.1)])
    res, cnt = serving.simulate(a, 1, 1, 2, [4096, 4096], reqs, n, [0.01] * n, pair_capacity=[64, 64],
                                need_pairs=[350, 350, 10, 10])
    assert cnt["regrown"] == 1 and cnt["redone"] == 2
    assert not res["status"].any()
    assert a.stats()["n_live"] == 0


def test_simulate_rejects_bad_traces():
    vy, serving = _vy()
    a = serving.Arena(1 << 20, base=FAKE_BASE)
    reqs, n = _trace(serving, [(0, 1.0), (0, 0.5)])
    with pytest.raises(vy.VoyagerError):                   # arrivals out of order
        serving.simulate(a, 1, 1, 1, [100], reqs, n, [1.0, 1.0])
    reqs, n = _trace(serving, [(1, 0.0)])
    with pytest.raises(vy.VoyagerError):                   # no such session
        serving.simulate(a, 1, 1, 1, [100], reqs, n, [1.0])
    reqs, n = _trace(serving, [(0, 0.0)])
    with pytest.raises(vy.VoyagerError) as e:              # can never fit
        serving.simulate(a, 1, 1, 1, [2 << 20], reqs, n, [1.0])
    assert e.value.code == vy.VY_ERR_CAPACITY
    with pytest.raises(vy.VoyagerError):
        serving.simulate(a, 0, 1, 1, [100], reqs, n, [1.0])


def test_session_bytes_rejects_invalid():
    vy, serving = _vy()
    assert serving.session_bytes(serving.session_struct(None, 64, 64)) == 0


# ---------------------------------------------------------------- layouts ----

def test_struct_layouts_match_the_header(tmp_path):
    """sizeof / offsetof of the serving structs as a C compiler lays them out,
    against the binding's ctypes structures."""
    vy, serving = _vy()
    src = tmp_path / "layout.c"
    fields = {
        "vy_session": ["scene", "width", "height", "tau", "alpha_filter", "max_gaussians", "max_pairs"],
        "vy_frame_req": ["session", "reserved", "t_arrival", "cam", "image"],
        "vy_frame_stats": ["image_hash", "n_cut", "n_pairs", "n_visible", "flags", "n_frontier", "reserved"],
        "vy_frame_result": ["t_admit", "t_dispatch", "t_start", "t_done", "status", "stream"],
        "vy_server_config": ["arena", "n_streams", "streams", "max_inflight", "max_viewers", "max_batch", "reserved",
                             "batch_gaussians", "batch_pairs"],
        "vy_camera": ["R", "pos", "fx", "fy", "cx", "cy", "width", "height", "znear"],
        "vy_view": ["scene", "cut", "cam", "image"],
        "vy_render_opts": ["alpha_filter", "bg", "save_state", "split_min_pairs", "walk", "lut_entries", "band_jobs"],
        "vy_grads": ["mean", "log_scale", "quat", "opacity_logit", "sh", "mean2d", "quat_raw"],
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "vy_serve.h"', "int main(void) {"]
    for s, fs in fields.items():
        lines.append(f'  printf("{s} %zu\\n", sizeof({s}));')
        for f in fs:
            lines.append(f'  printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    lines.append("  return 0;\n}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    c = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    for s, fs in fields.items():
        cls = getattr(vy, s)
        assert int(c[s]) == ctypes.sizeof(cls), s
        for f in fs:
            assert int(c[f"{s}.{f}"]) == getattr(cls, f).offset, (s, f)


# ------------------------------------------------------------ walkthrough ----

def _walk_call(vy, n_frames, depth, cuts, ctxs, streams, images, scene=FAKE_BASE, mode=0):
    """vy_walkthrough with stand-in handles: every call here must fail (or
    return) in the argument checks, before any handle is used."""
    P = ctypes.c_void_p
    cams = (vy.vy_camera * max(1, n_frames))()
    arr = lambda xs: (P * max(1, len(xs)))(*xs) if xs is not None else None
    return vy.lib().vy_walkthrough(P(scene) if scene else None, cams, n_frames, 2.0, mode, None, None, depth,
                                   arr(cuts), arr(ctxs), arr(streams), arr(images),
                                   len(images) if images is not None else 0, None, None, None)


def test_walkthrough_argument_checks():
    vy, _ = _vy()
    c, x, s, im = [FAKE_BASE + 16 * k for k in range(8)], [FAKE_BASE + 4096 + 16 * k for k in range(8)], \
        [FAKE_BASE + 8192 + 16 * k for k in range(8)], [FAKE_BASE + 65536 * (k + 1) for k in range(8)]
    E = vy.VY_ERR_ARG
    assert _walk_call(vy, 4, 2, c[:2], x[:2], s[:2], im[:2], scene=0) == E            # no scene
    assert _walk_call(vy, -1, 2, c[:2], x[:2], s[:2], im[:2]) == E                     # negative count
    assert _walk_call(vy, 4, 0, c[:2], x[:2], s[:2], im[:2]) == E                      # depth 0
    assert _walk_call(vy, 4, 17, c * 3, x * 3, s * 3, im[:1] * 17) == E                # depth above 16
    assert _walk_call(vy, 4, 2, [c[0], c[0]], x[:2], s[:2], im[:2]) == E               # a cut twice
    assert _walk_call(vy, 4, 2, c[:2], [x[1], x[1]], s[:2], im[:2]) == E               # a context twice
    assert _walk_call(vy, 4, 2, c[:2], x[:2], [s[0], s[0]], im[:2]) == E               # a stream twice
    assert _walk_call(vy, 4, 2, c[:2], x[:2], s[:2], im[:3]) == E                      # 3 images, 2 slots
    assert _walk_call(vy, 4, 2, c[:2], x[:2], s[:2], [im[0], 0]) == E                  # a NULL image
    assert _walk_call(vy, 4, 2, c[:2], x[:2], None, im[:2]) == E                       # no streams
    assert "depth" in vy.lib().vy_last_error().decode() or "distinct" in vy.lib().vy_last_error().decode()
    assert _walk_call(vy, 4, 2, c[:2], x[:2], s[:2], im[:2], mode=1 << 10) == E        # unknown mode bit
    assert _walk_call(vy, 0, 2, c[:2], x[:2], s[:2], im[:2], mode=vy.VY_WALK_FULL_EACH | vy.VY_CUT_DFS) == vy.VY_OK
    # nothing to render: returns before touching any handle or stream
    assert _walk_call(vy, 0, 3, c[:3], x[:3], s[:3], im[:6]) == vy.VY_OK
