"""Multi-viewer serving on top of the per-frame path (vy_serve.h).

Owners for the serving entry points (argument marshalling only; admission,
scheduling and every frame run in the library), the seeded multi-viewer
workload, and the serving benchmark:

    python -m paper_2506_02774_amd.serving [--viewers 64] [--seconds 4] ...

Workload: several resident city scenes of the same leaf density, viewer
sessions on them at mixed resolutions, each asking for frames as a Poisson
process (30 Hz by default) along the scene's street-level walkthrough path.
Every viewer keeps its previous cut (the temporal search's state) and its
render buffers resident while its session lasts.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import sys
import time

import numpy as np

from . import (VY_ERR_ARG, VY_RUN_REALTIME, VoyagerError, check, lib, make_camera, vy_frame_req,
               vy_frame_result, vy_frame_stats, vy_server_config, vy_session)

RESOLUTIONS = {"360p": (640, 360), "720p": (1280, 720), "1080p": (1920, 1080)}

RESULT_DTYPE = np.dtype([("t_admit", "f8"), ("t_dispatch", "f8"), ("t_start", "f8"), ("t_done", "f8"),
                         ("status", "i4"), ("stream", "i4")])
STATS_DTYPE = np.dtype([("image_hash", "u8"), ("n_cut", "u4"), ("n_pairs", "u4"), ("n_visible", "u4"),
                        ("flags", "u4"), ("n_frontier", "u4"), ("reserved", "u4")])
assert RESULT_DTYPE.itemsize == ctypes.sizeof(vy_frame_result)
assert STATS_DTYPE.itemsize == ctypes.sizeof(vy_frame_stats)


class Arena:
    """A device range (torch uint8 tensor) managed by a vy_arena."""

    def __init__(self, nbytes: int, device="cuda", base=None):
        L = lib()
        if base is None:
            import torch
            self.mem = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
            base = self.mem.data_ptr()
        else:                      # a caller-owned range (the arena never touches it)
            self.mem = None
        h = ctypes.c_void_p()
        check(L.vy_arena_create(ctypes.c_void_p(int(base)), int(nbytes), ctypes.byref(h)), "vy_arena_create")
        self.handle = h
        self.base, self.nbytes = int(base), int(nbytes)

    def alloc(self, nbytes: int) -> int:
        p = ctypes.c_void_p()
        check(lib().vy_arena_alloc(self.handle, int(nbytes), ctypes.byref(p)), "vy_arena_alloc")
        return int(p.value)

    def release(self, ptr: int):
        check(lib().vy_arena_release(self.handle, ctypes.c_void_p(int(ptr))), "vy_arena_release")

    def stats(self):
        u, lf = ctypes.c_size_t(), ctypes.c_size_t()
        nl, nf = ctypes.c_int64(), ctypes.c_int64()
        check(lib().vy_arena_stats(self.handle, ctypes.byref(u), ctypes.byref(lf), ctypes.byref(nl),
                                   ctypes.byref(nf)), "vy_arena_stats")
        return dict(used=u.value, largest_free=lf.value, n_live=nl.value, n_free_blocks=nf.value)

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().vy_arena_free(self.handle)
                self.handle = None
        except Exception:
            pass


def session_struct(scene, width, height, tau=2.0, alpha_filter=True, max_gaussians=0, max_pairs=0) -> vy_session:
    s = vy_session()
    s.scene = scene.handle if scene is not None else None
    s.width, s.height = int(width), int(height)
    s.tau = float(tau)
    s.alpha_filter = 1 if alpha_filter else 0
    s.max_gaussians, s.max_pairs = int(max_gaussians), int(max_pairs)
    return s


def session_bytes(sess: vy_session) -> int:
    return int(lib().vy_session_bytes(ctypes.byref(sess)))


def build_requests(reqs) -> ctypes.Array:
    """reqs: iterable of (session, t_arrival, camera, image_ptr or 0)."""
    reqs = list(reqs)
    arr = (vy_frame_req * max(1, len(reqs)))()
    for i, (s, t, cam, img) in enumerate(reqs):
        q = arr[i]
        q.session = int(s)
        q.reserved = 0
        q.t_arrival = float(t)
        if cam is not None:
            q.cam = make_camera(cam)
        q.image = int(img) if img else None
    return arr, len(reqs)


def _config(arena: Arena, n_streams, stream_ptrs, max_inflight, max_viewers, max_batch=0, batch_gaussians=0,
            batch_pairs=0):
    c = vy_server_config()
    c.arena = arena.handle
    c.n_streams = int(n_streams)
    c.streams = stream_ptrs
    c.max_inflight = int(max_inflight)
    c.max_viewers = int(max_viewers)
    c.max_batch = int(max_batch)
    c.reserved = 0
    c.batch_gaussians = int(batch_gaussians)
    c.batch_pairs = int(batch_pairs)
    return c


def batch_capacity(max_batch):
    """Capacities of a stream's batch context for max_batch frames of the
    serving workload: 3.5e6 cut Gaussians and 8e6 pairs per frame (above the
    largest measured, an 18M-leaf scene at 1920x1080)."""
    return min(max_batch * 3_500_000, 0x7FFFFFFF), min(max_batch * 8_000_000, 0x7FFFFFFF)


class Server:
    """vy_server over an arena and `n_streams` torch streams of default
    priority; max_batch > 1 fuses the frames dispatched to a stream in one
    scheduling pass into one batched render (vy_render_batch)."""

    def __init__(self, arena: Arena, n_streams=4, max_inflight=2, max_viewers=64, max_batch=0, batch_gaussians=0,
                 batch_pairs=0):
        import torch
        L = lib()
        self.arena = arena
        self.streams = [torch.cuda.Stream() for _ in range(int(n_streams))]
        self._ptrs = (ctypes.c_void_p * len(self.streams))(*[s.cuda_stream for s in self.streams])
        bg, bp = batch_capacity(max_batch) if max_batch > 1 else (0, 0)
        bg, bp = batch_gaussians or bg, batch_pairs or bp
        self.config = _config(arena, len(self.streams), ctypes.cast(self._ptrs, ctypes.POINTER(ctypes.c_void_p)),
                              max_inflight, max_viewers, max_batch, bg, bp)
        h = ctypes.c_void_p()
        check(L.vy_server_create(ctypes.byref(self.config), ctypes.byref(h)), "vy_server_create")
        self.handle = h

    def run(self, sessions, reqs, n_reqs, realtime=True, stats=True):
        """Serves the trace; returns (results numpy [n], stats numpy [n] or None)."""
        import torch
        L = lib()
        sess_arr = (vy_session * max(1, len(sessions)))(*sessions)
        res = (vy_frame_result * max(1, n_reqs))()
        st = torch.empty((max(1, n_reqs), 4), dtype=torch.int64, device="cuda") if stats else None
        torch.cuda.synchronize()       # the caller's device work (uploads, buffers) is done first
        rc = L.vy_server_run(self.handle, sess_arr, len(sessions), reqs, int(n_reqs),
                             VY_RUN_REALTIME if realtime else 0,
                             ctypes.c_void_p(st.data_ptr()) if st is not None else None, res)
        check(rc, "vy_server_run")
        out = np.frombuffer(bytes(res), dtype=RESULT_DTYPE)[:n_reqs].copy()
        stv = None
        if st is not None:
            torch.cuda.synchronize()
            stv = np.frombuffer(st.cpu().numpy().tobytes(), dtype=STATS_DTYPE)[:n_reqs].copy()
        return out, stv

    def last_run(self):
        a, w, p, g, r = (ctypes.c_int64() for _ in range(5))
        b = ctypes.c_size_t()
        check(lib().vy_server_last_run(self.handle, ctypes.byref(a), ctypes.byref(w), ctypes.byref(p),
                                       ctypes.byref(b), ctypes.byref(g), ctypes.byref(r)), "vy_server_last_run")
        return dict(admitted=a.value, waited=w.value, peak_resident=p.value, peak_bytes=b.value, regrown=g.value,
                    redone=r.value)

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().vy_server_free(self.handle)
                self.handle = None
        except Exception:
            pass


def simulate(arena: Arena, n_streams, max_inflight, max_viewers, session_bytes_list, reqs, n_reqs, service_s,
             realtime=True, pair_capacity=None, need_pairs=None):
    """vy_server_simulate: the server's policy against a model of the GPU (no GPU needed)."""
    L = lib()
    cfg = _config(arena, n_streams, None, max_inflight, max_viewers)
    ns = max(1, len(session_bytes_list))
    sb = (ctypes.c_int64 * ns)(*[int(b) for b in session_bytes_list])
    pc = (ctypes.c_int64 * ns)(*[int(b) for b in pair_capacity]) if pair_capacity is not None else None
    sv = (ctypes.c_double * max(1, n_reqs))(*[float(x) for x in service_s])
    npairs = (ctypes.c_uint32 * max(1, n_reqs))(*[int(x) for x in need_pairs]) if need_pairs is not None else None
    res = (vy_frame_result * max(1, n_reqs))()
    cnt = (ctypes.c_int64 * 6)()
    check(L.vy_server_simulate(ctypes.byref(cfg), sb, pc, len(session_bytes_list), reqs, int(n_reqs), sv, npairs,
                               VY_RUN_REALTIME if realtime else 0, res, cnt), "vy_server_simulate")
    out = np.frombuffer(bytes(res), dtype=RESULT_DTYPE)[:n_reqs].copy()
    return out, dict(admitted=cnt[0], waited=cnt[1], peak_resident=cnt[2], peak_bytes=cnt[3], regrown=cnt[4],
                     redone=cnt[5])


# ----------------------------------------------------------------------------
# Workload
# ----------------------------------------------------------------------------

def make_trace(scene_cfgs, n_seats=64, seconds=4.0, rate_hz=30.0, resolutions=("360p", "720p", "1080p"),
               frames=(45, 135), gap_s=0.25, seed=3000, yaw_jitter_deg=30.0):
    """Seeded viewer sessions and their frame requests.

    Every seat runs sessions back to back until `seconds`: a session picks a
    scene and a resolution uniformly, a length in frames uniformly in
    `frames`, a start index on the scene's walkthrough path and a heading
    offset; its frames arrive as a Poisson process of `rate_hz`; the next
    session of the seat starts an exponential gap (mean `gap_s`) after the
    last frame. Returns (sessions, requests): sessions as dicts (scene index,
    width, height), requests as (session, t_arrival, camera), by arrival."""
    import scenegen
    rng = np.random.default_rng(seed)
    paths = [scenegen.walkthrough_path(c) for c in scene_cfgs]
    sessions, reqs = [], []
    for seat in range(n_seats):
        t = rng.uniform(0.0, 0.1)
        while t < seconds:
            si = int(rng.integers(len(scene_cfgs)))
            res = resolutions[int(rng.integers(len(resolutions)))]
            W, H = RESOLUTIONS[res]
            n = int(rng.integers(frames[0], frames[1] + 1))
            pos, yaw = paths[si]
            n = min(n, len(yaw))
            off = int(rng.integers(0, len(yaw) - n + 1))
            dyaw = math.radians(rng.uniform(-yaw_jitter_deg, yaw_jitter_deg))
            sid = len(sessions)
            sessions.append(dict(scene=si, width=W, height=H, res=res, seat=seat, frames=n))
            for j in range(n):
                cam = scenegen.look_camera(pos[off + j], yaw[off + j] + dyaw, 0.0, W, H, scene_cfgs[si].fov_x_deg)
                reqs.append((sid, t, cam))
                t += rng.exponential(1.0 / rate_hz)
            t += rng.exponential(gap_s)
    order = sorted(range(len(reqs)), key=lambda i: (reqs[i][1], i))
    return sessions, [reqs[i] for i in order]


def latency_summary(res, arrivals=None):
    """Frames per second over the run; with arrivals, the latency from arrival
    to the end of the frame's last kernel (p50, p99, max)."""
    t0 = min(float(arrivals.min()) if arrivals is not None else 0.0, float(res["t_start"].min()))
    span = float(res["t_done"].max()) - t0
    out = dict(frames=int(len(res)), fps=round(len(res) / span, 1), makespan_s=round(span, 4),
               gpu_ms_mean=round(float(np.mean(res["t_done"] - res["t_start"])) * 1e3, 4))
    if arrivals is not None:
        lat = (res["t_done"] - arrivals) * 1e3
        out.update(p50_ms=round(float(np.percentile(lat, 50)), 3), p99_ms=round(float(np.percentile(lat, 99)), 3),
                   max_ms=round(float(lat.max()), 3))
    return out


def log(msg):
    print(f"[serving {time.perf_counter() - _T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


_T0 = time.perf_counter()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--viewers", type=int, default=64, help="seats: viewers served at once")
    ap.add_argument("--seconds", type=float, default=4.0, help="length of the arrival trace")
    ap.add_argument("--rate", type=float, default=30.0, help="frame requests per second per viewer")
    ap.add_argument("--leaves", default="1000000,4000000,8000000,18000000", help="leaves of the resident scenes")
    ap.add_argument("--tau", type=float, default=2.0)
    ap.add_argument("--modes", default="1x1,8x2,2x16b8,4x16b8",
                    help="server shapes to compare, STREAMSxINFLIGHT[bBATCH]; the first is the one-at-a-time "
                         "baseline; bBATCH fuses up to BATCH frames per stream into one batched render")
    ap.add_argument("--sustainable-rate", type=float, default=15.0,
                    help="a second, lighter trace (frame requests per second per viewer) that the one-at-a-time "
                         "baseline can keep up with, for the latency comparison")
    ap.add_argument("--budget-gib", type=float, default=160.0, help="device memory for resident viewers")
    ap.add_argument("--seed", type=int, default=3000)
    args = ap.parse_args(argv)
    import torch
    import scenegen
    from . import Scene

    cfgs = []
    for n in [int(x) for x in args.leaves.split(",")]:
        cfgs.append(scenegen.CONFIGS["full"] if n == scenegen.CONFIGS["full"].n_leaf
                    else scenegen.scaled_config("full", n))
    scenes = []
    for c in cfgs:
        log(f"scene {c.name}: {c.n_leaf} leaves")
        scenes.append(Scene(scenegen.make_city(c)))
        scenes[-1].host = None                      # the host copy is not needed any more
    node_bytes = sum(s.ws.numel() + s.arrays["sh"].numel() * 4 for s in scenes)
    sessions, trace = make_trace(cfgs, args.viewers, args.seconds, args.rate, seed=args.seed)
    log(f"{len(sessions)} sessions, {len(trace)} frame requests over {args.seconds:g} s "
        f"({args.viewers} viewers at {args.rate:g} Hz); scenes hold {node_bytes / 2**30:.1f} GiB")
    sess = [session_struct(scenes[s["scene"]], s["width"], s["height"], args.tau, True) for s in sessions]
    need = [session_bytes(s) for s in sess]
    arena = Arena(int(args.budget_gib * 2**30))
    reqs, n = build_requests((s, t, cam, 0) for (s, t, cam) in trace)
    arrivals = np.array([t for (_, t, _) in trace])
    # the lighter trace: same seats and scenes, fewer requests per second
    sessions_l, trace_l = make_trace(cfgs, args.viewers, args.seconds, args.sustainable_rate, seed=args.seed + 1)
    sess_l = [session_struct(scenes[s["scene"]], s["width"], s["height"], args.tau, True) for s in sessions_l]
    reqs_l, n_l = build_requests((s, t, cam, 0) for (s, t, cam) in trace_l)
    arrivals_l = np.array([t for (_, t, _) in trace_l])
    log(f"lighter trace: {len(sessions_l)} sessions, {n_l} frame requests at {args.sustainable_rate:g} Hz per viewer "
        f"({n_l / args.seconds:.0f} requests/s offered)")

    modes = []
    for m in args.modes.split(","):
        m = m.lower()
        batch = 0
        if "b" in m:
            m, b = m.split("b")
            batch = int(b)
        ns, inflight = (int(x) for x in m.split("x"))
        name = f"streams={ns},inflight={inflight}" + (f",batch={batch}" if batch > 1 else "")
        modes.append((name, ns, inflight, batch))
    px = np.array([sessions[q]["width"] * sessions[q]["height"] for (q, _, _) in trace], np.float64)
    out = dict(viewers=args.viewers, sessions=len(sessions), frames=n, seconds=args.seconds, rate_hz=args.rate,
               scenes=[c.n_leaf for c in cfgs], scene_gib=round(node_bytes / 2**30, 2), tau=args.tau,
               resolutions=sorted({s["res"] for s in sessions}), budget_gib=args.budget_gib,
               session_mib_mean=round(float(np.mean(need)) / 2**20, 1), baseline=modes[0][0], modes={})
    out["sustainable_trace"] = dict(rate_hz=args.sustainable_rate, sessions=len(sessions_l), frames=n_l,
                                    offered_fps=round(n_l / args.seconds, 1))
    hashes = {}
    for name, ns, inflight, batch in modes:
        srv = Server(arena, ns, inflight, args.viewers, batch)
        row = {}
        for key in ("saturated", "realtime", "realtime_sustainable"):
            realtime = key != "saturated"
            light = key == "realtime_sustainable"
            res, st = srv.run(sess_l if light else sess, reqs_l if light else reqs, n_l if light else n,
                              realtime=realtime, stats=True)
            row[key] = latency_summary(res, (arrivals_l if light else arrivals) if realtime else None)
            row[key]["frame_errors"] = int(np.count_nonzero(res["status"] != 0))
            row[key]["frames_flagged"] = {k: int(np.count_nonzero(st["flags"] & b))
                                          for k, b in (("pairs", 1), ("cut", 2), ("render_wait", 4), ("cut_wait", 8))}
            row[key].update(srv.last_run())
            if not light:
                hashes[(name, key)] = st["image_hash"].copy()
            log(f"{name} {key}: {row[key]}")
            if "per_pixel" not in out:
                # cut and pair counts per pixel, by scene and resolution
                rows = {}
                for si, c in enumerate(cfgs):
                    for r in sorted(RESOLUTIONS):
                        m = np.array([sessions[q]["scene"] == si and sessions[q]["res"] == r for (q, _, _) in trace])
                        if m.any():
                            rows[f"{c.n_leaf // 1000000}M/{r}"] = dict(
                                frames=int(m.sum()), cut_p50=int(np.percentile(st["n_cut"][m], 50)),
                                cut_max=int(st["n_cut"][m].max()),
                                pairs_per_px_p50=round(float(np.percentile(st["n_pairs"][m] / px[m], 50)), 3),
                                pairs_per_px_max=round(float(np.max(st["n_pairs"][m] / px[m])), 3))
                out["per_pixel"] = rows
                log(f"cut and pairs by scene/resolution: {rows}")
        out["modes"][name] = row
        del srv
    base = out["modes"][modes[0][0]]["saturated"]["fps"]
    for name, _, _, _ in modes:
        out["modes"][name]["saturated"]["speedup_vs_baseline"] = round(out["modes"][name]["saturated"]["fps"] / base, 3)
    ref = hashes[(modes[0][0], "saturated")]
    out["images_identical_across_modes"] = bool(all(np.array_equal(ref, h) for h in hashes.values()))
    log(f"images identical across modes: {out['images_identical_across_modes']}")
    print(json.dumps(out))
    return out


if __name__ == "__main__":
    main()
