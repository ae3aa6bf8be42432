#!/usr/bin/env python3
"""Walkthrough benchmark of the Voyager per-frame hot path on one MI355X.

A step is one frame: the LoD cut (temporal search seeded with the previous
frame's frontier, or a full search) followed by rendering (projection, binning
with or without the preemptive alpha filter, sort, blend). The default
workload is the city-scale walkthrough: 1.8e7 leaf Gaussians (3.6e7 hierarchy
nodes), 1920x1080, 300 frames, tau = 2 px, seeded synthetic scene and path.

Prints ONE JSON line: FPS of temporal LoD + alpha filter (the method) as
rendered by the walkthrough renderer (vy_walkthrough: --depth frames in flight
on as many streams, every image bitwise that of the one-at-a-time loop), with
p50/p99 frame times (GPU time from a frame's search to the end of its
rendering), the plain full-search + unfiltered renderer on the same frames
and in the same way, the same two with one frame in flight, the frames-in-
flight sweep, the 2x2 ablation for tau in {1, 2, 4} (one frame in flight),
bitwise gates (temporal cut == full cut, filtered image == unfiltered image,
walkthrough renderer == frame loop, every frame), per-stage times,
the roofline of the dominant kernel and each stage's fraction of the HBM
peak, the FP64 oracle (cut + sampled tiles of three frames at every tau,
compared with the GPU, and timed on 16 host threads and on one), the LUT
exponential of Section 4.2 (FPS and PSNR / SSIM against the exact image for
table sizes 8..128), and the plain renderer's own workload (2e6 leaves,
1280x720, 120 frames, full search + unfiltered, gated every frame and
compared with the oracle on every tenth). Then, in a child process once the walkthrough's buffers are freed, the
multi-viewer serving benchmark (paper_2506_02774_amd.serving: 64 viewers on 4
resident scenes at mixed resolutions, one frame at a time against several
streams); its JSON is embedded under "serving". Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (counts packed FP32 instructions)
FP32_UNPACKED_PEAK_TFLOPS = 78.6  # the same without packed FP32 (256 CUs x 4 SIMD x 16 lanes x 2 x 2.4 GHz)
# algorithmic work of the blend: 10 vector operations per pixel evaluation of a
# tile-list entry (offset 2, rho 5, clamp 1, pixel-box tests 2) plus one
# exponential per evaluation that reaches it; the blended contributions are a
# lower bound of the latter (each needed its exponential)
BLEND_OPS_EVAL, BLEND_OPS_EXP = 10.0, 1.0
ORACLE_THREADS = 16   # host threads for the oracle (the CPU share of one GPU on the box)
T0 = time.time()


def log(msg):
    print(f"[bench {time.time() - T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300, help="timed frames (the walkthrough length)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="full", help="tiny | med | full")
    ap.add_argument("--tau", type=float, default=2.0, help="tau of the headline number")
    ap.add_argument("--no-ablation", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the multi-viewer serving benchmark")
    ap.add_argument("--no-lut", action="store_true", help="skip the LUT-exponential study")
    ap.add_argument("--no-backward", action="store_true", help="skip timing the backward pass")
    ap.add_argument("--cpu-tiles", type=int, default=16, help="tiles the oracle renders per sampled frame")
    ap.add_argument("--oracle-frames", type=int, default=3, help="frames per tau compared with the oracle")
    ap.add_argument("--no-med", action="store_true", help="skip the 2M-leaf 720p plain-renderer workload")
    ap.add_argument("--max-pairs", type=int, default=96 << 20)
    ap.add_argument("--copy-mib", type=int, default=1024, help="size of the HBM copy used as the traffic reference")
    ap.add_argument("--depth", type=int, default=4, help="frames in flight of the headline walkthrough")
    ap.add_argument("--walk-depths", default="1,2,3,4", help="frames in flight swept for the walkthrough table")
    return ap.parse_args()


def frame_loop(vy, torch, scene, cams, tau, temporal, filt, state, full_cut, ctx, img, per_frame=True, lut=0,
               mode=0):
    """Run the frames; returns per-frame ms (events on torch's current stream)."""
    ev = []
    for i, cam in enumerate(cams):
        if per_frame:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
        if temporal:
            if i == 0:
                vy.vy_lod_cut(scene, cam, tau, out=state, mode=mode)
            else:
                vy.vy_lod_cut(scene, cam, tau, prev=state, out=state, mode=mode)
            cut = state
        else:
            vy.vy_lod_cut(scene, cam, tau, out=full_cut, mode=mode)
            cut = full_cut
        vy.vy_render(scene, cut, cam, ctx, image=img, alpha_filter=filt, lut_entries=lut)
        if per_frame:
            e1.record()
            ev.append((e0, e1))
    return ev


def timed(vy, torch, scene, cams, tau, temporal, filt, state, full_cut, ctx, img, lut=0, mode=0):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev = frame_loop(vy, torch, scene, cams, tau, temporal, filt, state, full_cut, ctx, img, lut=lut, mode=mode)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    rc, npairs, nvis = ctx.status()
    vy.check(rc, "vy_render_status")
    return dict(fps=len(cams) / wall, ms_per_step=1e3 * wall / len(cams), p50_ms=float(np.percentile(ms, 50)),
                p99_ms=float(np.percentile(ms, 99)), p99_ms_frames_1_on=float(np.percentile(ms[1:], 99))
                if len(ms) > 1 else float(ms[0]), mean_event_ms=float(ms.mean()))


def make_slots(vy, torch, scene, W, H, max_pairs, n):
    """Per-slot state of the walkthrough renderer: a cut, a render context, a
    stream and an image for each of n frames in flight. The first slot runs
    on the caller's stream: HIP gives a process 4 hardware queues by default,
    so 4 frames in flight then use exactly the 4 queues (a fifth stream would
    share one and serialise with it)."""
    return dict(cuts=[vy.Cut(scene) for _ in range(n)],
                ctxs=[vy.RenderContext(scene.n, W, H, max_pairs) for _ in range(n)],
                streams=[torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(n - 1)],
                images=[torch.empty((3, H, W), dtype=torch.float32, device="cuda") for _ in range(n)])


def walk_timed(vy, torch, scene, cams, tau, slots, depth, temporal=True, filt=True, passes=1):
    """vy_walkthrough over the path with `depth` frames in flight: throughput
    from the wall clock of a pass over all frames (the fastest of `passes`);
    per-frame GPU time (search start to render end, HIP events on the frame's
    stream) and the per-frame records (no capacity or wait flag on any frame)
    from a further pass."""
    from paper_2506_02774_amd.serving import STATS_DTYPE
    mode = 0 if temporal else vy.VY_WALK_FULL_EACH
    a = (scene, cams, tau, slots["cuts"][:depth], slots["ctxs"][:depth], slots["images"][:depth])
    kw = dict(streams=slots["streams"][:depth], mode=mode, alpha_filter=filt)
    wall = float("inf")
    for _ in range(passes):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vy.vy_walkthrough(*a, **kw)
        torch.cuda.synchronize()
        wall = min(wall, time.perf_counter() - t0)
    st = torch.zeros((len(cams), 4), dtype=torch.int64, device="cuda")
    ms = vy.vy_walkthrough(*a, stats=st, frame_ms=True, **kw)
    flags = np.frombuffer(st.cpu().numpy().tobytes(), dtype=STATS_DTYPE)["flags"]
    if flags.any():
        raise RuntimeError(f"walkthrough depth {depth}: {int((flags != 0).sum())} frames flagged (capacity or wait)")
    return dict(fps=len(cams) / wall, ms_per_step=1e3 * wall / len(cams), p50_ms=float(np.percentile(ms, 50)),
                p99_ms=float(np.percentile(ms, 99)), p99_ms_frames_1_on=float(np.percentile(ms[1:], 99))
                if len(ms) > 1 else float(ms[0]), mean_event_ms=float(ms.mean()))


def stage_bytes(stage, c):
    """Algorithmic HBM bytes of one frame's launches of `stage` (from counts)."""
    F, C, V, P, T, N, px = c["F"], c["C"], c["V"], c["P"], c["tiles"], c["N"], c["px"]
    return {
        "lod_classify": (4 + 32 + 16) * F + 4 * (F + C),
        "lod_compact": 2 * (N / 8) + 4 * (F + C),
        "lod_flat": 32 * N + 16 * N + N / 4,
        "blend_plan": 8 * T + 4 * T,
        "project": (4 + 48 + 192 + 68) * C,
        "depth_sort": 60 * C,
        "emit": (4 + 16 + 4) * V + 8 * P,
        "tile_sort": 32 * P,
        "ranges": 4 * P + 8 * T,
        "blend": (4 + 48) * P + 8 * T + 12 * px,
    }.get(stage, 0.0)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the per-frame path is measured on exactly one MI355X; several GPUs would "
                                   "take independent viewers, or screen-space bands of one frame, each",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import scenegen
    import paper_2506_02774_amd as vy
    if not os.path.exists(vy.LIB_PATH):
        from paper_2506_02774_amd import build as _b
        _b.build(force=True)
    vy.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    cfg = scenegen.CONFIGS[args.config]
    K, W = args.steps, args.warmup
    log(f"generating scene '{cfg.name}' ({cfg.n_leaf} leaves)")
    host = scenegen.make_city(cfg)
    log(f"scene: {host.n_nodes} nodes, {len(host.level_start) - 1} levels; uploading")
    scene = vy.Scene(host)
    nbad = scene.validate()
    assert nbad == 0, f"scene validation failed: {nbad}"
    cams = scenegen.walkthrough(cfg, frames=K)
    warm = scenegen.walkthrough(cfg, seed=cfg.path_seed + 100, frames=max(W, 1))
    Wd, Hd = cfg.width, cfg.height
    ctx = vy.RenderContext(scene.n, Wd, Hd, args.max_pairs)
    state, full_cut, aux = vy.Cut(scene), vy.Cut(scene), vy.Cut(scene)
    img = torch.empty((3, Hd, Wd), dtype=torch.float32, device="cuda")
    img2 = torch.empty_like(img)
    ntiles = ((Wd + 15) // 16) * ((Hd + 15) // 16)
    log(f"GPU memory in use: {torch.cuda.memory_allocated() / 2**30:.1f} GiB")
    # reference copy of known size (HBM-to-HBM): its achieved rate is the practical
    # bandwidth ceiling, and under rocprofv3 --pmc its FETCH/WRITE_SIZE calibrate the counters
    nb = args.copy_mib << 20
    src = torch.empty(nb // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    # an elementwise kernel (x * 1) rather than copy_, which may go to the runtime's blit path
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    ce0, ce1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ce0.record()
    for _ in range(5):
        torch.mul(src, 1.0, out=dst)
    ce1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * nb * 5 / (ce0.elapsed_time(ce1) * 1e-3) / 1e9
    del src, dst
    log(f"reference copy {args.copy_mib} MiB: {copy_gbs:.0f} GB/s (read + write)")
    peaks = vy.measure_peaks()
    log(f"measured vector peaks: FP32 FMA {peaks['fma_fp32_tflops']:.1f} TFLOP/s (no packed FP32), "
        f"v_exp_f32 {peaks['exp_f32_gops']:.0f} G/s")

    # ---------------------------------------------------------------- warmup
    for temporal, filt in ((True, True), (False, False)):
        frame_loop(vy, torch, scene, warm[:W] if W else warm[:1], args.tau, temporal, filt, state, full_cut, ctx,
                   img, per_frame=False)
    torch.cuda.synchronize()
    rc, np_w, nv_w = ctx.status()
    vy.check(rc, "warmup")
    log("warmup done")

    # ------------------------------------------------------------ headline
    # one frame at a time (a host loop over vy_lod_cut + vy_render on one stream)
    seq = timed(vy, torch, scene, cams, args.tau, True, True, state, full_cut, ctx, img)
    log(f"one frame in flight, temporal + alpha filter: {seq['fps']:.1f} FPS, p50 {seq['p50_ms']:.3f} ms, "
        f"p99 {seq['p99_ms']:.3f} ms")
    seq_base = timed(vy, torch, scene, cams, args.tau, False, False, state, full_cut, ctx, img)
    log(f"one frame in flight, full + unfiltered: {seq_base['fps']:.1f} FPS, p50 {seq_base['p50_ms']:.3f} ms, "
        f"p99 {seq_base['p99_ms']:.3f} ms")
    # the walkthrough renderer: frames in flight on several streams (vy_walkthrough)
    depths = sorted({int(d) for d in args.walk_depths.split(",") if d} | {args.depth})
    slots = make_slots(vy, torch, scene, Wd, Hd, args.max_pairs, max(depths))
    # warm-up on the path itself, so that every slot's buffers have been touched at full size
    for filt in (True, False):
        vy.vy_walkthrough(scene, cams, args.tau, slots["cuts"], slots["ctxs"], slots["images"],
                          streams=slots["streams"], alpha_filter=filt)
    torch.cuda.synchronize()
    walk = {}
    for d in depths:   # the sweep: fastest of two passes per depth
        walk[d] = walk_timed(vy, torch, scene, cams, args.tau, slots, d, passes=2)
        log(f"walkthrough, {d} frame(s) in flight, temporal + alpha filter: {walk[d]['fps']:.1f} FPS, "
            f"frame p50 {walk[d]['p50_ms']:.3f} ms, p99 {walk[d]['p99_ms']:.3f} ms")
    # the headline and its plain-renderer baseline: one timed pass of the K frames each
    head = walk_timed(vy, torch, scene, cams, args.tau, slots, args.depth)
    base = walk_timed(vy, torch, scene, cams, args.tau, slots, args.depth, temporal=False, filt=False)
    log(f"walkthrough, {args.depth} frame(s) in flight, full + unfiltered: {base['fps']:.1f} FPS, "
        f"frame p50 {base['p50_ms']:.3f} ms, p99 {base['p99_ms']:.3f} ms")
    log(f"temporal + alpha filter: {head['fps']:.1f} FPS, p50 {head['p50_ms']:.3f} ms, p99 {head['p99_ms']:.3f} ms")

    # ------------------------------------------------------------ ablation
    ablation = {}
    if not args.no_ablation:
        for tau in cfg.taus:
            row = {}
            for temporal in (False, True):
                for filt in (False, True):
                    r = timed(vy, torch, scene, cams, tau, temporal, filt, state, full_cut, ctx, img)
                    row[("temporal" if temporal else "full") + ("+filter" if filt else "")] = {
                        k: round(v, 4) for k, v in r.items() if k in ("fps", "p50_ms", "p99_ms")}
            ablation[f"tau={tau:g}"] = row
            log(f"ablation tau={tau:g}: " + ", ".join(f"{k} {v['fps']:.0f}" for k, v in row.items()))

    # --------- LoD traversal: workgroup breadth-first (default), per-thread depth-first,
    # and the subtree-chunk traversal of Section 4.1 over the scene's partition
    traversal = {}
    t0p = time.perf_counter()
    scene.partition()
    torch.cuda.synchronize()
    traversal["partition_build_s"] = round(time.perf_counter() - t0p, 2)
    log(f"subtree partition built in {traversal['partition_build_s']} s")
    # the chunked searches give the default cut on every frame (temporal and full)
    chk = dict(frames=0, mismatch=0)
    a_cut, b_cut = vy.Cut(scene), vy.Cut(scene)
    for i, cam in enumerate(cams):
        vy.vy_lod_cut(scene, cam, args.tau, prev=a_cut if i else None, out=a_cut, mode=vy.VY_CUT_CHUNKED)
        vy.vy_lod_cut(scene, cam, args.tau, out=b_cut)
        fa, fb = a_cut.ids(), b_cut.ids()
        chk["mismatch"] += 0 if (np.array_equal(fa[0], fb[0]) and np.array_equal(fa[1], fb[1])) else 1
        if i % 10 == 0:
            fc = vy.vy_lod_cut(scene, cam, args.tau, out=b_cut, mode=vy.VY_CUT_CHUNKED).ids()
            chk["mismatch"] += 0 if (np.array_equal(fc[0], fb[0]) and np.array_equal(fc[1], fb[1])) else 1
        chk["frames"] += 1
    del a_cut, b_cut
    traversal["chunked_equals_default"] = chk
    log(f"chunked traversal == default: {chk}")
    for name, temporal, filt in (("temporal+filter", True, True), ("full+unfiltered", False, False)):
        row = {}
        for tname, mode in (("bfs", 0), ("dfs", vy.VY_CUT_DFS), ("chunked", vy.VY_CUT_CHUNKED)):
            r = timed(vy, torch, scene, cams, args.tau, temporal, filt, state, full_cut, ctx, img, mode=mode)
            vy.profile_begin(64 * K + 64)
            frame_loop(vy, torch, scene, cams, args.tau, temporal, filt, state, full_cut, ctx, img, per_frame=False,
                       mode=mode)
            torch.cuda.synchronize()
            pr = vy.profile_end()
            row[tname] = {"fps": round(r["fps"], 2), "p99_ms": round(r["p99_ms"], 4),
                          "lod_ms_per_frame": round(sum(ms for k, (ms, n) in pr.items() if k.startswith("lod_")) / K,
                                                    5),
                          "lod_traverse_ms_per_frame": round(pr["lod_traverse"][0] / K, 5)}
        traversal[name] = row
        log(f"traversal {name}: {row}")

    # ------------------------------------------------- LUT exponential (Eq. 5)
    lut = {} if args.no_lut else lut_study(vy, torch, scene, cams, args.tau, state, full_cut, ctx, img, img2)

    # ------------------------------------------------ gates + per-frame counts
    log("verification pass (temporal cut == full cut, filtered == unfiltered, every frame at every tau; "
        "walkthrough renderer == frame loop at the headline tau)")
    gates = dict(frames=0, cut_mismatch=0, image_mismatch=0, walkthrough_image_mismatch=0)
    # every frame of the headline configuration, each into its own image
    walk_imgs = [torch.empty((3, Hd, Wd), dtype=torch.float32, device="cuda")
                 for _ in range(-(-K // args.depth) * args.depth)]
    vy.vy_walkthrough(scene, cams, args.tau, slots["cuts"][:args.depth], slots["ctxs"][:args.depth], walk_imgs,
                      streams=slots["streams"][:args.depth], alpha_filter=True)
    torch.cuda.synchronize()
    gates_tau = {}
    avg = None
    tst = vy.Cut(scene)
    for tau in sorted(set(cfg.taus) | {args.tau}):
        head_tau = tau == args.tau
        g = dict(frames=0, cut_mismatch=0, image_mismatch=0)
        counts = dict(F=0.0, C=0.0, V=0.0, P=0.0, P_unf=0.0, evals=0.0, contribs=0.0)
        for i, cam in enumerate(cams):
            vy.vy_lod_cut(scene, cam, tau, prev=tst if i else None, out=tst)
            vy.vy_lod_cut(scene, cam, tau, out=full_cut)
            nf_t, nc_t = tst.counts()
            nf_f, nc_f = full_cut.counts()
            same = (nf_t, nc_t) == (nf_f, nc_f)
            if same:
                pt = [ctypes_ptr(vy, tst, k) for k in (0, 1)]
                pf = [ctypes_ptr(vy, full_cut, k) for k in (0, 1)]
                same = bool(torch.equal(vy.device_view(pt[0], (nf_t,)), vy.device_view(pf[0], (nf_f,)))) and \
                    bool(torch.equal(vy.device_view(pt[1], (nc_t,)), vy.device_view(pf[1], (nc_f,))))
            g["cut_mismatch"] += 0 if same else 1
            vy.vy_render(scene, full_cut, cam, ctx, image=img, alpha_filter=False)
            rc, p_unf, _ = ctx.status()
            vy.check(rc)
            vy.vy_render(scene, tst, cam, ctx, image=img2, alpha_filter=True, save_state=head_tau)
            rc, p_f, v_f = ctx.status()
            vy.check(rc)
            if head_tau:
                _, Nc, Ne = ctx.saved(Wd, Hd, evals=True)
                counts["evals"] += float(Ne[Ne >= 0].sum())
                counts["contribs"] += float(Nc.sum())
                if not torch.equal(walk_imgs[i].view(torch.int32), img2.view(torch.int32)):
                    gates["walkthrough_image_mismatch"] += 1
            if not torch.equal(img.view(torch.int32), img2.view(torch.int32)):
                g["image_mismatch"] += 1
            g["frames"] += 1
            counts["F"] += nf_t
            counts["C"] += nc_t
            counts["V"] += v_f
            counts["P"] += p_f
            counts["P_unf"] += p_unf
        nfr = max(1, g["frames"])
        gates_tau[f"tau={tau:g}"] = dict(g, mean_counts={k: round(v / nfr) for k, v in counts.items()
                                                         if k not in ("evals", "contribs") or head_tau})
        for k in ("frames", "cut_mismatch", "image_mismatch"):
            gates[k] += g[k]
        if head_tau:
            avg = {k: v / nfr for k, v in counts.items()}
        log(f"gates tau={tau:g}: {g}")
    del walk_imgs
    gates["per_tau"] = gates_tau
    log(f"gates: {gates}; mean |F| {avg['F']:.0f} |C| {avg['C']:.0f} visible {avg['V']:.0f} "
        f"pairs {avg['P']:.0f} (unfiltered {avg['P_unf']:.0f})")

    # ------------------------------------------------------- stage profile
    prof = {}
    for name, temporal, filt in (("temporal+filter", True, True), ("full", False, False)):
        vy.profile_begin(64 * K + 64)
        frame_loop(vy, torch, scene, cams, args.tau, temporal, filt, state, full_cut, ctx, img, per_frame=False)
        torch.cuda.synchronize()
        prof[name] = vy.profile_end()
    stages = prof["temporal+filter"]
    log("stage ms/frame (temporal+filter): " + ", ".join(
        f"{k} {ms / K:.3f}" for k, (ms, n) in stages.items() if n))
    cnt = dict(F=avg["F"], C=avg["C"], V=avg["V"], P=avg["P"], tiles=ntiles, N=scene.n, px=Wd * Hd, filter=True)
    per_stage = {}
    for k, (ms, n) in stages.items():
        if not n:
            continue
        b = stage_bytes(k, cnt)
        gbs = b / (ms / K * 1e-3) / 1e9 if ms > 0 and b > 0 else None
        per_stage[k] = dict(ms_per_frame=round(ms / K, 5), launches_per_frame=n / K,
                            algorithmic_bytes_per_frame=round(b) if b > 0 else None,
                            algorithmic_GBps=round(gbs, 1) if gbs else None,
                            frac_of_hbm_peak=round(gbs / HBM_PEAK_GBS, 4) if gbs else None)
    dom = max(((k, ms) for k, (ms, n) in stages.items() if n), key=lambda t: t[1])[0]
    bwd = None if args.no_backward else backward_study(vy, torch, scene, cams, args.tau, state, ctx, img)
    dom_ms, dom_n = stages[dom]
    launch_ms = dom_ms / dom_n
    traffic = read_traffic(dom)
    if dom == "blend":
        # ALU-bound kernel: algorithmic vector operations from the per-pixel evaluation counts
        ops = BLEND_OPS_EVAL * avg["evals"] + BLEND_OPS_EXP * avg["contribs"]
        ops_per_launch = ops * K / dom_n
        achieved = ops_per_launch / (launch_ms * 1e-3) / 1e12
        roofline = dict(kernel="blend_jobs<true,false,false,false>", bound="alu", achieved=round(achieved, 3),
                        peak=FP32_VECTOR_PEAK_TFLOPS, unit="TFLOP/s", frac=round(achieved / FP32_VECTOR_PEAK_TFLOPS, 5),
                        traffic=traffic, peak_unpacked=FP32_UNPACKED_PEAK_TFLOPS,
                        frac_of_unpacked=round(achieved / FP32_UNPACKED_PEAK_TFLOPS, 5),
                        peak_measured=round(peaks["fma_fp32_tflops"], 2),
                        frac_of_measured=round(achieved / peaks["fma_fp32_tflops"], 5),
                        launch_ms=round(launch_ms, 5), ops_per_launch=round(ops_per_launch),
                        ops_formula="10 * evals + contribs (exponentials, lower bound)",
                        evals_per_launch=round(avg["evals"]), contribs_per_launch=round(avg["contribs"]),
                        algorithmic_bytes_per_launch=round(stage_bytes("blend", cnt)),
                        hbm_frac=round(stage_bytes("blend", cnt) / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
        log(f"dominant kernel blend: {launch_ms:.4f} ms/launch, {achieved:.2f} T ops/s algorithmic")
    else:
        bytes_per_launch = stage_bytes(dom, cnt) * K / dom_n
        achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
        roofline = dict(kernel=dom, bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                        launch_ms=round(launch_ms, 5), bytes_per_launch=round(bytes_per_launch))
        log(f"dominant kernel {dom}: {launch_ms:.4f} ms/launch, {achieved:.0f} GB/s algorithmic")

    # ------------------------------------------------------ oracle on CPU
    cpu = None
    parity = dict(gates)
    if not args.no_cpu_baseline:
        cpu, par = oracle_leg(vy, torch, host, scene, cams, cfg.taus, args.tau, ctx, img, full_cut, args.cpu_tiles,
                              args.oracle_frames)
        parity.update(par)
    med = None
    if not args.no_med and args.config == "full":
        med = med_study(vy, torch, args)
    train = None
    if not args.no_backward and args.config == "full":
        train = train_study(vy, torch)

    out = {
        "metric": "FPS, 18M-Gaussian 1080p walkthrough (temporal vs full LoD); p99 frame ms",
        "value": round(head["fps"], 2), "unit": "FPS", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(head["ms_per_step"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"city-{cfg.name}: {cfg.n_leaf} leaves ({scene.n} nodes), {Wd}x{Hd}, "
                               f"{K}-frame walkthrough, tau={args.tau:g} px, temporal LoD + alpha filter, "
                               f"{args.depth} frames in flight",
                   "leaves": cfg.n_leaf, "nodes": scene.n, "width": Wd, "height": Hd, "frames": K, "tau": args.tau,
                   "frames_in_flight": args.depth},
        "p50_ms": round(head["p50_ms"], 4), "p99_ms": round(head["p99_ms"], 4),
        "p99_ms_frames_1_on": round(head["p99_ms_frames_1_on"], 4),
        "full_unfiltered": {k: round(v, 4) for k, v in base.items()},
        "speedup_vs_full_unfiltered": round(head["fps"] / base["fps"], 3),
        "one_frame_in_flight": {"temporal+filter": {k: round(v, 4) for k, v in seq.items()},
                                "full+unfiltered": {k: round(v, 4) for k, v in seq_base.items()},
                                "speedup": round(seq["fps"] / seq_base["fps"], 3)},
        "walkthrough_frames_in_flight": {str(d): {k: round(v, 4) for k, v in r.items() if k != "ms_per_step"}
                                         for d, r in walk.items()},
        "ablation": ablation,
        "lut": lut,
        "lod_traversal": traversal,
        "backward": bwd,
        "mean_counts": {k: round(v) for k, v in avg.items()},
        "stages": per_stage,
        "stages_full_unfiltered_ms_per_frame": {k: round(ms / K, 5) for k, (ms, n) in prof["full"].items() if n},
        "roofline": roofline,
        "reference_copy_GBps": round(copy_gbs, 1),
        "measured_peaks": {"fma_fp32_tflops": round(peaks["fma_fp32_tflops"], 2),
                           "exp_f32_gops": round(peaks["exp_f32_gops"], 1), "copy_GBps": round(copy_gbs, 1)},
        "cpu_baseline": cpu,
        "parity": parity,
        "med_plain_renderer": med,
        "training_500k_720p": train,
    }
    if not args.no_serving and args.config == "full":
        del ctx, state, full_cut, img, scene, slots
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        out["serving"] = serving_child()
    print(json.dumps(out), flush=True)


def lut_study(vy, torch, scene, cams, tau, state, full_cut, ctx, img, img2, ms=(8, 16, 32, 64, 128),
              frames=(0, 60, 120, 180, 240, 299)):
    """The LUT exponential of Section 4.2 on the walkthrough (temporal cut + alpha
    filter): FPS per table size m, and PSNR / SSIM of its images against the
    exact exponential's on sampled frames (filtered == unfiltered checked there)."""
    from paper_2506_02774_amd import quality
    exact = timed(vy, torch, scene, cams, tau, True, True, state, full_cut, ctx, img)
    out = {"exact": {"fps": round(exact["fps"], 2), "p50_ms": round(exact["p50_ms"], 4)}}
    frames = [f for f in frames if f < len(cams)]
    refs = {}
    for f in frames:
        vy.vy_lod_cut(scene, cams[f], tau, out=full_cut)
        vy.vy_render(scene, full_cut, cams[f], ctx, image=img, alpha_filter=True)
        refs[f] = img.cpu().numpy()
    for m in ms:
        r = timed(vy, torch, scene, cams, tau, True, True, state, full_cut, ctx, img, lut=m)
        ps, ss, mismatch = [], [], 0
        for f in frames:
            vy.vy_lod_cut(scene, cams[f], tau, out=full_cut)
            vy.vy_render(scene, full_cut, cams[f], ctx, image=img, alpha_filter=True, lut_entries=m)
            vy.vy_render(scene, full_cut, cams[f], ctx, image=img2, alpha_filter=False, lut_entries=m)
            mismatch += 0 if torch.equal(img.view(torch.int32), img2.view(torch.int32)) else 1
            a = img.cpu().numpy()
            ps.append(quality.psnr(a, refs[f]))
            ss.append(quality.ssim(a, refs[f]))
        out[f"m={m}"] = {"fps": round(r["fps"], 2), "p50_ms": round(r["p50_ms"], 4),
                         "psnr_db_vs_exact": round(float(np.mean(ps)), 2), "ssim_vs_exact": round(float(np.mean(ss)), 5),
                         "filtered_ne_unfiltered_frames": mismatch}
        log(f"LUT m={m}: {out[f'm={m}']}")
    return out


def backward_study(vy, torch, scene, cams, tau, state, ctx, img, n_frames=60):
    """Forward with saved state, then the backward of sum(w * image) (w fixed,
    seeded), frame after frame on the walkthrough: per-stage milliseconds and
    the rate of forward + backward steps. Gradient buffers for every node are
    allocated once; each backward overwrites the rows of the cut's Gaussians."""
    import ctypes
    L = vy.lib()
    n = scene.n
    shapes = dict(mean=(n, 3), log_scale=(n, 3), quat=(n, 4), opacity_logit=(n,), sh=(n, 48))
    gt = {k: torch.zeros(sh, device="cuda") for k, sh in shapes.items()}
    g = vy.vy_grads()
    for k, t in gt.items():
        setattr(g, k, t.data_ptr())
    gen = torch.Generator(device="cuda").manual_seed(5)
    w = torch.randn(img.shape, device="cuda", generator=gen)
    frames = cams[:n_frames]
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def step(i, cam):
        if i == 0:
            vy.vy_lod_cut(scene, cam, tau, out=state)
        else:
            vy.vy_lod_cut(scene, cam, tau, prev=state, out=state)
        vy.vy_render(scene, state, cam, ctx, image=img, alpha_filter=True, save_state=True)
        c = vy.make_camera(cam)
        vy.check(L.vy_render_backward(scene.handle, state.handle, ctypes.byref(c), ctypes.c_void_p(w.data_ptr()),
                                      ctypes.byref(g), ctx.handle, stream), "vy_render_backward")

    step(0, frames[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, cam in enumerate(frames):
        step(i, cam)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    vy.profile_begin(64 * len(frames) + 64)
    for i, cam in enumerate(frames):
        step(i, cam)
    torch.cuda.synchronize()
    prof = vy.profile_end()
    K = len(frames)
    fwd_ms = sum(ms for k, (ms, nl) in prof.items() if nl and not k.startswith("bwd_")) / K
    out = {"frames": K, "steps_per_s": round(K / wall, 2), "ms_per_step": round(1e3 * wall / K, 4),
           "forward_saved_ms": round(fwd_ms, 4),
           "bwd_blend_ms": round(prof["bwd_blend"][0] / K, 4), "bwd_project_ms": round(prof["bwd_project"][0] / K, 4),
           "grad_norms_last_frame": {k: float(t.norm()) for k, t in gt.items()}}
    log(f"backward: {out}")
    return out


def train_study(vy, torch, target_cut=500_000, iters=20, warm=3):
    """The differentiable rendering workload: a cut of about 500,000 Gaussians
    taken from the 2e6-leaf city at 1280x720 (street level at a corner of the
    city looking across it; tau found by bisection), whose Gaussians become
    the leaves of a training tree rendered at tau = 0; a target image rendered
    from parameters perturbed by N(0, 0.01) in position and colour (SH) and
    N(0, 0.05) in log-scale and opacity logit; the loss L1 + 0.2 (1 - SSIM).
    One iteration: repack the parameters, render with saved state, the loss,
    its backward (the hand-written adjoint behind the autograd function, then
    the SSIM's), and an Adam step. Reports ms per iteration (HIP events
    around each part, and the wall clock)."""
    import scenegen
    from paper_2506_02774_amd import training
    cfg = scenegen.CONFIGS["med"]
    log("training: generating the 2e6-leaf city")
    host = scenegen.make_city(cfg)
    W, H = cfg.width, cfg.height
    e = 0.95 * cfg.extent / 2
    cam = scenegen.look_camera([-e, -e, cfg.eye], math.atan2(e, e), 0.0, W, H, cfg.fov_x_deg)
    probe = vy.Scene(host)
    lo, hi, n_cut = 0.5, 64.0, 0
    cut = vy.Cut(probe)
    for _ in range(40):            # the cut shrinks as tau grows
        tau = math.sqrt(lo * hi)
        n_cut = vy.vy_lod_cut(probe, cam, tau, out=cut).counts()[1]
        if abs(n_cut - target_cut) <= 0.005 * target_cut:
            break
        lo, hi = (tau, hi) if n_cut > target_cut else (lo, tau)
    _, C = cut.ids()
    del probe, cut
    sub = dict(mean=host.mean[C], log_scale=host.log_scale[C], quat=host.quat[C],
               opacity_logit=host.opacity_logit[C], sh=host.sh[C])
    tree = scenegen.build_hierarchy(sub)
    r = training.Renderer(tree, W, H, tau=0.0, alpha_filter=True, max_pairs=16 << 20)
    params = r.parameters_from(tree)
    gen = torch.Generator(device="cuda").manual_seed(4)
    with torch.no_grad():
        pert = {k: v.detach().clone() for k, v in params.items()}
        pert["mean"] += 0.01 * torch.randn(pert["mean"].shape, device="cuda", generator=gen)
        pert["sh"] += 0.01 * torch.randn(pert["sh"].shape, device="cuda", generator=gen)
        pert["log_scale"] += 0.05 * torch.randn(pert["log_scale"].shape, device="cuda", generator=gen)
        pert["opacity_logit"] += 0.05 * torch.randn(pert["opacity_logit"].shape, device="cuda", generator=gen)
        target = r(pert, cam).detach().clone()
    n_vis = r.ctx.status()[2]
    opt = torch.optim.Adam([params[k] for k in training.PARAMS], lr=1e-3)
    names = ("forward", "loss", "backward", "adam")
    ev = {k: [] for k in names}
    losses = []

    def one(record):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        e[0].record()
        img = r(params, cam)
        e[1].record()
        loss = training.loss_l1_ssim(img, target)
        e[2].record()
        opt.zero_grad(set_to_none=True)
        loss.backward()
        e[3].record()
        opt.step()
        e[4].record()
        if record:
            for i, k in enumerate(names):
                ev[k].append((e[i], e[i + 1]))
        return loss

    for _ in range(warm):
        one(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        losses.append(one(True))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in ev.items()}
    out = dict(workload=f"city-med: {cfg.n_leaf} leaves, a cut of {n_cut} Gaussians (tau={tau:.3f} px) at {W}x{H} "
                        f"as the leaves of a training tree ({tree.n_nodes} nodes), target from perturbed parameters, "
                        f"L1 + 0.2 (1 - SSIM), Adam",
               cut_gaussians=int(n_cut), rendered_gaussians=int(r.cut.counts()[1]), projected_gaussians=int(n_vis),
               iters=iters,
               ms_per_iteration=round(1e3 * wall / iters, 4), iterations_per_s=round(iters / wall, 2),
               ms_parts={k: round(v, 4) for k, v in ms.items()},
               loss_first_last=[round(float(losses[0]), 6), round(float(losses[-1]), 6)])
    log(f"training: {out}")
    del r, params, pert, target, opt
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def serving_child(timeout_s=480):
    """Runs the serving benchmark in a child process (its progress goes to our
    stderr) and returns its JSON, or an error record."""
    import subprocess
    log("serving benchmark (child process)")
    try:
        r = subprocess.run([sys.executable, "-m", "paper_2506_02774_amd.serving"], cwd=ROOT, stdout=subprocess.PIPE,
                           timeout=timeout_s)
        lines = r.stdout.decode().strip().splitlines()
        if r.returncode != 0 or not lines:
            return {"error": f"exit status {r.returncode}"}
        return json.loads(lines[-1])
    except Exception as e:   # the walkthrough results above stand on their own
        return {"error": repr(e)}


def read_traffic(stage):
    """HBM traffic per launch of the dominant kernel from the committed PMC
    summary (profiles/*traffic*.md, a JSON line), or None when it is missing or
    was taken on a different version of the kernel source."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2506_02774_amd", "csrc", "render.hip")
    sha = hashlib.sha1(open(src, "rb").read()).hexdigest()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*traffic*.md"))):
        for line in open(f):
            line = line.strip()
            if line.startswith("{") and '"traffic_bytes_per_launch"' in line:
                d = json.loads(line)
                if d.get("stage") == stage and d.get("source_sha1") == sha:
                    return d["traffic_bytes_per_launch"]
    return None


def ctypes_ptr(vy, cut, which):
    import ctypes
    pf, pc, pn = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    vy.check(vy.lib().vy_cut_arrays(cut.handle, ctypes.byref(pf), ctypes.byref(pc), ctypes.byref(pn)))
    return (pf.value, pc.value)[which]


def oracle_frame(vy, torch, host, scene, cam, tau, ctx, img, cut, n_tiles, threads, seed=7):
    """One frame against the FP64 oracle: the GPU's full-search cut against the
    brute force over every node, and n_tiles 16x16 tiles of its image (the two
    with the longest tile lists, where the work concentrates, and random ones)
    against the oracle's per-pixel blend of the GPU's cut. Returns the parity
    record and the oracle's seconds per part."""
    from oracle import lod as olod, project as oproj, render as orender
    W, H = cam.width, cam.height
    tx_n, ty_n = (W + 15) // 16, (H + 15) // 16
    t0 = time.perf_counter()
    F_or, C_or, P = olod.cut_bruteforce(host, cam, tau, threads=threads)
    t_cut = time.perf_counter() - t0
    vy.vy_lod_cut(scene, cam, tau, out=cut)
    F, C = cut.ids()
    cmp = olod.compare_cut(host, cam, tau, F, C, oracle=(F_or, C_or, P))
    del P
    vy.vy_render(scene, cut, cam, ctx, image=img, alpha_filter=True)
    rc, n_pairs, _ = ctx.status()
    vy.check(rc)
    keys, vals, ranges = ctx.pairs(W, H)
    length = ranges[:, 1].astype(np.int64) - ranges[:, 0]
    gimg = img.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(seed)
    heavy = {int(t) for t in np.argsort(-length)[:2]}
    rest = [t for t in rng.permutation(tx_n * ty_n).tolist() if t not in heavy][:max(0, n_tiles - len(heavy))]
    tiles = sorted(heavy | set(rest))
    t0 = time.perf_counter()
    proj = oproj.project_threaded(host, C, cam, threads=threads)
    t_proj = time.perf_counter() - t0
    t0 = time.perf_counter()
    ref = orender.render_image(proj, W, H, tiles=tiles, threads=threads)
    t_tiles = time.perf_counter() - t0
    mask = ~np.isnan(ref["image"][0])
    err = np.abs(gimg - np.nan_to_num(ref["image"]))[:, mask]
    amb = ref["ambiguous"][mask]
    max_err = float(err[:, ~amb].max()) if (~amb).any() else 0.0
    rec = dict(tau=tau, cut_ok=bool(cmp["ok"]), cut_near_threshold=cmp["expand_diff"], C=int(len(C)),
               tiles=len(tiles), tile_pairs_max=int(length.max()), px=int(mask.sum()), max_abs=round(max_err, 6),
               mean_abs=float(err.mean()), ambiguous_px=int(amb.sum()),
               image_ok=bool(max_err <= 2e-3 and float(err.mean()) <= 1e-4))
    secs = dict(cut=t_cut, project=t_proj, tiles=t_tiles, n_tiles=len(tiles), all_tiles=tx_n * ty_n,
                n_nodes=host.n_nodes, n_cut=int(len(C)))
    return rec, secs


def oracle_leg(vy, torch, host, scene, cams, taus, head_tau, ctx, img, cut, n_tiles, n_frames):
    """The FP64 oracle on the host: parity on n_frames frames spread over the
    walkthrough at every tau (cut + sampled tiles), timed on ORACLE_THREADS
    threads; and one frame at the headline tau on a single thread. Returns
    (cpu_baseline record, parity record)."""
    from threadpoolctl import threadpool_limits
    K = len(cams)
    frames = sorted({int(round(x)) for x in np.linspace(0, K - 1, max(1, n_frames))})
    recs, timing = [], None
    with threadpool_limits(limits=1):       # one BLAS thread per oracle thread
        for tau in sorted(set(taus) | {head_tau}):
            for f in frames:
                rec, secs = oracle_frame(vy, torch, host, scene, cams[f], tau, ctx, img, cut, n_tiles,
                                         ORACLE_THREADS, seed=7 + f)
                rec["frame"] = f
                recs.append(rec)
                log(f"oracle tau={tau:g} frame {f}: {rec}")
                if tau == head_tau and f == frames[0]:
                    timing = secs
        one, one_secs = oracle_frame(vy, torch, host, scene, cams[0], head_tau, ctx, img, cut, 4, 1, seed=99)

    def frame_s(t):
        return t["cut"] + t["project"] + t["tiles"] * t["all_tiles"] / t["n_tiles"]

    def sample(t, threads):
        return (f"frame 0, tau={head_tau:g}: brute-force cut over all {t['n_nodes']} nodes ({t['cut']:.1f}s), "
                f"projection of {t['n_cut']} cut Gaussians ({t['project']:.1f}s), {t['n_tiles']} of "
                f"{t['all_tiles']} tiles blended ({t['tiles']:.1f}s), scaled to a whole frame; FP64 numpy on "
                f"{threads} host thread(s)")

    cpu = dict(value=round(1.0 / frame_s(timing), 6), unit="FPS", cores=ORACLE_THREADS, kind="oracle",
               sample=sample(timing, ORACLE_THREADS),
               seconds=round(timing["cut"] + timing["project"] + timing["tiles"], 2),
               single_core=dict(value=round(1.0 / frame_s(one_secs), 6), unit="FPS", cores=1,
                                sample=sample(one_secs, 1),
                                seconds=round(one_secs["cut"] + one_secs["project"] + one_secs["tiles"], 2)))
    par = dict(oracle_frames=recs, oracle_cut_ok=all(r["cut_ok"] for r in recs),
               oracle_image_ok=all(r["image_ok"] for r in recs),
               oracle_max_abs=max(r["max_abs"] for r in recs), oracle_mean_abs_max=max(r["mean_abs"] for r in recs),
               oracle_single_core_frame=dict(one, frame=0))
    log(f"cpu baseline: {cpu['value']:.5f} FPS on {ORACLE_THREADS} threads, {cpu['single_core']['value']:.5f} "
        f"FPS on one; oracle cut ok {par['oracle_cut_ok']}, image ok {par['oracle_image_ok']}")
    return cpu, par


def med_study(vy, torch, args, tau=2.0, oracle_every=10, tiles_per_frame=4):
    """The plain renderer's own workload: 2e6 leaves (about 4e6 nodes),
    1280x720, the 120-frame walkthrough, tau = 2, full LoD search each frame
    and no alpha filter, one frame at a time; beside it the temporal search +
    filter on the same frames. Gates every frame (temporal cut == full cut,
    filtered image == unfiltered image) and compares frames 0, 10, ..., 110
    with the oracle (cut + sampled tiles)."""
    import scenegen
    from threadpoolctl import threadpool_limits
    cfg = scenegen.CONFIGS["med"]
    log(f"med: generating scene ({cfg.n_leaf} leaves)")
    host = scenegen.make_city(cfg)
    scene = vy.Scene(host)
    assert scene.validate() == 0
    cams = scenegen.walkthrough(cfg)
    warm = scenegen.walkthrough(cfg, seed=cfg.path_seed + 100, frames=5)
    W, H = cfg.width, cfg.height
    ctx = vy.RenderContext(scene.n, W, H, 32 << 20)
    state, full_cut = vy.Cut(scene), vy.Cut(scene)
    img = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
    img2 = torch.empty_like(img)
    for temporal, filt in ((False, False), (True, True)):
        frame_loop(vy, torch, scene, warm, tau, temporal, filt, state, full_cut, ctx, img, per_frame=False)
    torch.cuda.synchronize()
    plain = timed(vy, torch, scene, cams, tau, False, False, state, full_cut, ctx, img)
    method = timed(vy, torch, scene, cams, tau, True, True, state, full_cut, ctx, img)
    log(f"med: plain renderer (full + unfiltered) {plain['fps']:.1f} FPS p99 {plain['p99_ms']:.3f} ms; "
        f"temporal + filter {method['fps']:.1f} FPS p99 {method['p99_ms']:.3f} ms")
    g = dict(frames=0, cut_mismatch=0, image_mismatch=0)
    for i, cam in enumerate(cams):
        vy.vy_lod_cut(scene, cam, tau, prev=state if i else None, out=state)
        vy.vy_lod_cut(scene, cam, tau, out=full_cut)
        Ft, Ct = state.ids()
        Ff, Cf = full_cut.ids()
        g["cut_mismatch"] += 0 if (np.array_equal(Ft, Ff) and np.array_equal(Ct, Cf)) else 1
        vy.vy_render(scene, full_cut, cam, ctx, image=img, alpha_filter=False)
        vy.check(ctx.status()[0])
        vy.vy_render(scene, state, cam, ctx, image=img2, alpha_filter=True)
        vy.check(ctx.status()[0])
        g["image_mismatch"] += 0 if torch.equal(img.view(torch.int32), img2.view(torch.int32)) else 1
        g["frames"] += 1
    recs = []
    with threadpool_limits(limits=1):
        for f in range(0, len(cams), oracle_every):
            rec, _ = oracle_frame(vy, torch, host, scene, cams[f], tau, ctx, img, full_cut, tiles_per_frame,
                                  ORACLE_THREADS, seed=50 + f)
            rec["frame"] = f
            recs.append(rec)
    out = dict(workload=f"city-med: {cfg.n_leaf} leaves ({scene.n} nodes), {W}x{H}, {len(cams)}-frame walkthrough, "
                        f"tau={tau:g} px, one frame in flight",
               plain_full_unfiltered={k: round(v, 4) for k, v in plain.items()},
               temporal_filter={k: round(v, 4) for k, v in method.items()},
               speedup=round(method["fps"] / plain["fps"], 3), gates=g,
               oracle_frames=recs, oracle_cut_ok=all(r["cut_ok"] for r in recs),
               oracle_image_ok=all(r["image_ok"] for r in recs),
               oracle_max_abs=max(r["max_abs"] for r in recs))
    log(f"med: gates {g}; oracle cut ok {out['oracle_cut_ok']}, image ok {out['oracle_image_ok']} "
        f"(max abs {out['oracle_max_abs']})")
    del ctx, state, full_cut, img, img2, scene
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
