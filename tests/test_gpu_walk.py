"""GPU checks of the walkthrough renderer (vy_walkthrough in vy_serve.h,
through the C ABI): with 1, 2 or 3 frames in flight every cut and image is
bitwise the one of a loop over vy_lod_cut + vy_render, split calls continue
from `prev`, the per-frame records match the images, errors stop the call
cleanly, and one frame against the oracle."""
import numpy as np
import pytest

import scenegen
from oracle import project as oproj, render as orender

from gpu_util import image_parity, require_gpu

pytestmark = pytest.mark.gpu

W, H = 200, 120   # not a multiple of 16


def host_hash(img):
    """Sum over i of SplitMix64's finaliser of (i << 32 | bits(img[i])), mod 2^64."""
    bits = np.ascontiguousarray(img, np.float32).view(np.uint32).ravel().astype(np.uint64)
    z = (np.arange(bits.size, dtype=np.uint64) << np.uint64(32)) | bits
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    z = z ^ (z >> np.uint64(31))
    return int(z.sum(dtype=np.uint64))


@pytest.fixture(scope="module")
def world(tiny_scene):
    vy = require_gpu()
    import torch
    cfg = scenegen.CONFIGS["tiny"]
    scene = vy.Scene(tiny_scene)
    pos, yaw = scenegen.walkthrough_path(cfg, frames=40)
    cams = [scenegen.look_camera(pos[j], yaw[j], 0.05, W, H) for j in range(14)]
    # the reference: one frame after the other with the plain entry points
    cut, ctx = vy.Cut(scene), vy.RenderContext(scene.n, W, H, 1 << 20)
    ref, ids = [], []
    for j, cam in enumerate(cams):
        vy.vy_lod_cut(scene, cam, 2.0, prev=cut if j else None, out=cut)
        ref.append(vy.vy_render(scene, cut, cam, ctx, alpha_filter=True).cpu().numpy())
        vy.check(ctx.status()[0])
        ids.append(cut.ids())
    torch.cuda.synchronize()
    return vy, torch, scene, cams, ref, ids, tiny_scene


def _slots(vy, torch, scene, depth):
    cuts = [vy.Cut(scene) for _ in range(depth)]
    ctxs = [vy.RenderContext(scene.n, W, H, 1 << 20) for _ in range(depth)]
    streams = [torch.cuda.Stream() for _ in range(depth)]
    return cuts, ctxs, streams


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_images_equal_frame_loop(world, depth):
    vy, torch, scene, cams, ref, ids, host = world
    from paper_2506_02774_amd.serving import STATS_DTYPE
    cuts, ctxs, streams = _slots(vy, torch, scene, depth)
    n = len(cams)
    images = [torch.full((3, H, W), float("nan"), device="cuda") for _ in range(n - n % depth)]
    images += [torch.full((3, H, W), float("nan"), device="cuda") for _ in range(depth)] if n % depth else []
    stats = torch.zeros((n, 4), dtype=torch.int64, device="cuda")
    ms = vy.vy_walkthrough(scene, cams, 2.0, cuts, ctxs, images, streams=streams, alpha_filter=True, stats=stats,
                           frame_ms=True)
    torch.cuda.synchronize()
    assert ms.shape == (n,) and np.all(ms > 0)
    st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=STATS_DTYPE)
    assert not st["flags"].any()
    for i in range(n):
        img = images[i % len(images)].cpu().numpy() if len(images) >= n else None
        if img is not None:
            assert np.array_equal(img.view(np.uint32), ref[i].view(np.uint32)), i
        assert st["image_hash"][i] == host_hash(ref[i]), i
        F, C = ids[i]
        assert st["n_cut"][i] == len(C) and st["n_frontier"][i] == len(F), i
    F, C = cuts[(n - 1) % depth].ids()
    assert np.array_equal(F, ids[-1][0]) and np.array_equal(C, ids[-1][1])


def test_reused_images_and_split_calls(world):
    """Two images per slot reused along the path, and the path cut in two
    calls: the second continues from the first one's last cut."""
    vy, torch, scene, cams, ref, ids, host = world
    depth = 2
    cuts, ctxs, streams = _slots(vy, torch, scene, depth)
    images = [torch.empty((3, H, W), device="cuda") for _ in range(2 * depth)]
    k = 7
    vy.vy_walkthrough(scene, cams[:k], 2.0, cuts, ctxs, images, streams=streams, alpha_filter=True)
    torch.cuda.synchronize()
    for i in range(k - len(images), k):
        assert np.array_equal(images[i % len(images)].cpu().numpy().view(np.uint32), ref[i].view(np.uint32)), i
    # continue: frame k starts from frame k-1's cut; prev is one of the slots' cuts
    stats = torch.zeros((len(cams) - k, 4), dtype=torch.int64, device="cuda")
    vy.vy_walkthrough(scene, cams[k:], 2.0, cuts, ctxs, images, streams=streams, prev=cuts[(k - 1) % depth],
                      alpha_filter=True, stats=stats)
    torch.cuda.synchronize()
    from paper_2506_02774_amd.serving import STATS_DTYPE
    st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=STATS_DTYPE)
    for j in range(len(cams) - k):
        assert st["image_hash"][j] == host_hash(ref[k + j]), k + j
    last = len(cams) - k - 1
    F, C = cuts[last % depth].ids()
    assert np.array_equal(C, ids[-1][1])


def test_error_stops_and_joins(world):
    """A camera larger than the contexts fails vy_render's check at that frame
    (before any launch): the call returns the error, the earlier frames
    complete and the caller's stream continues after them."""
    import ctypes
    vy, torch, scene, cams, ref, ids, host = world
    depth = 2
    cuts, ctxs, streams = _slots(vy, torch, scene, depth)
    big = scenegen.look_camera([0.0, 0.0, 20.0], 0.3, 0.0, W + 32, H)
    path = list(cams[:3]) + [big] + list(cams[3:5])
    images = [torch.full((3, H, W), float("nan"), device="cuda") for _ in range(2)]
    # the binding checks image shapes itself, so the C entry point is called directly
    P = ctypes.c_void_p
    cam_arr = (vy.vy_camera * len(path))(*[vy.make_camera(c) for c in path])
    o = vy.vy_render_opts()
    o.alpha_filter = 1
    torch.cuda.synchronize()
    rc = vy.lib().vy_walkthrough(scene.handle, cam_arr, len(path), 2.0, 0, ctypes.byref(o), None, depth,
                                 (P * 2)(*[c.handle for c in cuts]), (P * 2)(*[c.handle for c in ctxs]),
                                 (P * 2)(*[s.cuda_stream for s in streams]),
                                 (P * 2)(images[0].data_ptr(), images[1].data_ptr()), 2, None, None,
                                 P(torch.cuda.current_stream().cuda_stream))
    assert rc == vy.VY_ERR_ARG
    torch.cuda.synchronize()
    # frames 0..2 were rendered: frame 2 is in image 0 (slot 0), frame 1 in image 1
    assert np.array_equal(images[0].cpu().numpy().view(np.uint32), ref[2].view(np.uint32))
    assert np.array_equal(images[1].cpu().numpy().view(np.uint32), ref[1].view(np.uint32))


def test_full_search_each_frame(world):
    """VY_WALK_FULL_EACH: every frame a full search, unfiltered, the frames not
    chained: cuts and images equal the temporal loop's (the search and the
    filter change neither, bit for bit)."""
    vy, torch, scene, cams, ref, ids, host = world
    from paper_2506_02774_amd.serving import STATS_DTYPE
    depth = 3
    cuts, ctxs, streams = _slots(vy, torch, scene, depth)
    n = 9
    images = [torch.full((3, H, W), float("nan"), device="cuda") for _ in range(n)]
    stats = torch.zeros((n, 4), dtype=torch.int64, device="cuda")
    vy.vy_walkthrough(scene, cams[:n], 2.0, cuts, ctxs, images, streams=streams, mode=vy.VY_WALK_FULL_EACH,
                      alpha_filter=False, stats=stats)
    torch.cuda.synchronize()
    st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=STATS_DTYPE)
    for i in range(n):
        assert np.array_equal(images[i].cpu().numpy().view(np.uint32), ref[i].view(np.uint32)), i
        assert st["n_cut"][i] == len(ids[i][1]) and st["n_frontier"][i] == len(ids[i][0]), i
    F, C = cuts[(n - 1) % depth].ids()
    assert np.array_equal(F, ids[n - 1][0]) and np.array_equal(C, ids[n - 1][1])


def test_fewer_frames_than_slots(world):
    """Two frames with four slots: the unused slots' streams only join."""
    vy, torch, scene, cams, ref, ids, host = world
    cuts, ctxs, streams = _slots(vy, torch, scene, 4)
    images = [torch.full((3, H, W), float("nan"), device="cuda") for _ in range(4)]
    vy.vy_walkthrough(scene, cams[:2], 2.0, cuts, ctxs, images, streams=streams, alpha_filter=True)
    torch.cuda.synchronize()
    for i in range(2):
        assert np.array_equal(images[i].cpu().numpy().view(np.uint32), ref[i].view(np.uint32)), i
    assert np.isnan(images[2].cpu().numpy()).all() and np.isnan(images[3].cpu().numpy()).all()


def test_bad_arguments(world):
    vy, torch, scene, cams, ref, ids, host = world
    cuts, ctxs, streams = _slots(vy, torch, scene, 2)
    images = [torch.empty((3, H, W), device="cuda") for _ in range(3)]
    with pytest.raises(vy.VoyagerError) as e:      # 3 images for 2 slots
        vy.vy_walkthrough(scene, cams[:4], 2.0, cuts, ctxs, images, streams=streams)
    assert e.value.code == vy.VY_ERR_ARG
    with pytest.raises(vy.VoyagerError) as e:      # one stream twice
        vy.vy_walkthrough(scene, cams[:4], 2.0, cuts, ctxs, images[:2], streams=[streams[0], streams[0]])
    assert e.value.code == vy.VY_ERR_ARG
    with pytest.raises(vy.VoyagerError) as e:      # one cut twice
        vy.vy_walkthrough(scene, cams[:4], 2.0, [cuts[0], cuts[0]], ctxs, images[:2], streams=streams)
    assert e.value.code == vy.VY_ERR_ARG


def test_frame_matches_oracle(world):
    vy, torch, scene, cams, ref, ids, host = world
    cuts, ctxs, streams = _slots(vy, torch, scene, 2)
    images = [torch.empty((3, H, W), device="cuda") for _ in range(4)]
    vy.vy_walkthrough(scene, cams[:4], 2.0, cuts, ctxs, images, streams=streams, alpha_filter=True)
    torch.cuda.synchronize()
    F, C = cuts[1].ids()
    r = image_parity(images[3].cpu().numpy(), orender.render_image(oproj.project(host, C, cams[3]), W, H))
    assert r["ok"], r
