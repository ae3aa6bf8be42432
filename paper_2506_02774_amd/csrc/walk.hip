// Walkthrough renderer: the frames of one camera path with several frames in
// flight on several HIP streams.
//
// Frame i is exactly vy_lod_cut (the temporal search of Algorithm 1 seeded
// with frame i-1's cut) followed by vy_render. Only the searches form a chain:
// frame i's search needs frame i-1's frontier and nothing else, so frame i
// waits (one HIP event) for frame i-1's search, not for its rendering. The
// rendering of one frame then overlaps the search and the rendering of the
// next ones. That fills the GPU while the previous frame's last, longest blend
// jobs finish on a few compute units. Each frame keeps its own cut, render
// context and image slot (frame i uses slot i mod depth), and every launch of
// a slot goes to that slot's stream, so the work of one slot is ordered by its
// stream alone.
#include <cstring>
#include <vector>

#include "vy_common.hpp"
#include "../../include/vy_serve.h"

using namespace vy;

namespace {

constexpr int kMaxDepth = 16;

// HIP events created by one call, destroyed when it returns (HIP releases an
// event still pending once it completes).
struct EventSet {
  std::vector<hipEvent_t> ev;
  ~EventSet() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  int make(unsigned flags, hipEvent_t* out) {
    const hipError_t e = hipEventCreateWithFlags(out, flags);
    if (e != hipSuccess) return fail(VY_ERR_HIP, "vy_walkthrough: hipEventCreateWithFlags: %s", hipGetErrorString(e));
    ev.push_back(*out);
    return VY_OK;
  }
};

// n pairwise distinct entries, none NULL unless allowed (the null stream)
template <class T>
bool distinct(const T* const* a, int n, bool null_ok = false) {
  for (int i = 0; i < n; ++i) {
    if (!a[i] && !null_ok) return false;
    for (int j = 0; j < i; ++j)
      if (a[i] == a[j]) return false;
  }
  return true;
}

}  // namespace

extern "C" int vy_walkthrough(const vy_scene* scene, const vy_camera* cams, int64_t n_frames, float tau,
                              int32_t full_mode, const vy_render_opts* opts, vy_cut* prev, int32_t depth,
                              vy_cut* const* cuts, vy_render_ctx* const* ctxs, void* const* streams,
                              float* const* images, int64_t n_images, vy_frame_stats* stats, float* frame_ms,
                              void* stream) {
  if (!scene || n_frames < 0 || (n_frames > 0 && !cams))
    return fail(VY_ERR_ARG, "vy_walkthrough: bad scene, cameras or frame count");
  if (depth < 1 || depth > kMaxDepth) return fail(VY_ERR_ARG, "vy_walkthrough: depth %d not in 1..%d", depth, kMaxDepth);
  if (!cuts || !ctxs || !streams || !distinct(cuts, depth) || !distinct(ctxs, depth) ||
      !distinct((void* const*)streams, depth, true))
    return fail(VY_ERR_ARG, "vy_walkthrough: cuts, contexts and streams must be %d distinct handles each", depth);
  if (!images || n_images < 1 || n_images % depth != 0)
    return fail(VY_ERR_ARG, "vy_walkthrough: the number of images must be a positive multiple of depth");
  for (int64_t j = 0; j < n_images; ++j)
    if (!images[j]) return fail(VY_ERR_ARG, "vy_walkthrough: image %lld is NULL", (long long)j);
  if ((full_mode & ~(VY_CUT_FLAT | VY_CUT_DFS | VY_WALK_FULL_EACH)) != 0)
    return fail(VY_ERR_ARG, "vy_walkthrough: unknown mode %d", full_mode);
  if (n_frames == 0) return VY_OK;
  // frames in flight overlap: unless the caller chose, heavy tiles take the
  // band-job layout that spends the least work in all
  vy_render_opts ropts;
  memset(&ropts, 0, sizeof(ropts));
  if (opts) ropts = *opts;
  if (ropts.band_jobs == 0 && depth > 1) ropts.band_jobs = 2;
  // every frame searched from the root (no chain between frames), or the temporal chain
  const bool each_full = (full_mode & VY_WALK_FULL_EACH) != 0;
  const int cut_mode = full_mode & ~VY_WALK_FULL_EACH;

  hipStream_t caller = (hipStream_t)stream;
  EventSet es;
  hipEvent_t start, searched[2];
  int rc = es.make(hipEventDisableTiming, &start);
  for (int k = 0; k < 2 && rc == VY_OK; ++k) rc = es.make(hipEventDisableTiming, &searched[k]);
  std::vector<hipEvent_t> joined(depth), t0, t1;
  for (int k = 0; k < depth && rc == VY_OK; ++k) rc = es.make(hipEventDisableTiming, &joined[k]);
  if (frame_ms) {
    t0.resize(n_frames);
    t1.resize(n_frames);
    for (int64_t i = 0; i < n_frames && rc == VY_OK; ++i) {
      rc = es.make(hipEventDefault, &t0[i]);
      if (rc == VY_OK) rc = es.make(hipEventDefault, &t1[i]);
    }
  }
  if (rc != VY_OK) return rc;

  // every slot starts after the work already on the caller's stream
  if (stats) VY_HIP(hipMemsetAsync(stats, 0, sizeof(vy_frame_stats) * (size_t)n_frames, caller));
  VY_HIP(hipEventRecord(start, caller));
  for (int k = 0; k < depth; ++k) VY_HIP(hipStreamWaitEvent((hipStream_t)streams[k], start, 0));

  int err = VY_OK;
  for (int64_t i = 0; i < n_frames && err == VY_OK; ++i) {
    const int k = (int)(i % depth);
    hipStream_t st = (hipStream_t)streams[k];
    hipError_t he = hipSuccess;
    // the search of frame i starts from frame i-1's frontier (the event of the
    // previous search is recorded again only after this wait is enqueued)
    if (i > 0 && !each_full) he = hipStreamWaitEvent(st, searched[(i - 1) & 1], 0);
    if (he == hipSuccess && frame_ms) he = hipEventRecord(t0[i], st);
    if (he != hipSuccess) {
      err = fail(VY_ERR_HIP, "vy_walkthrough: frame %lld: %s", (long long)i, hipGetErrorString(he));
      break;
    }
    vy_cut* from = each_full ? nullptr : (i == 0 ? prev : cuts[(i - 1) % depth]);
    err = vy_lod_cut(scene, &cams[i], tau, from, cuts[k], cut_mode, st);
    if (err != VY_OK) break;
    he = hipEventRecord(searched[i & 1], st);
    if (he != hipSuccess) {
      err = fail(VY_ERR_HIP, "vy_walkthrough: frame %lld: %s", (long long)i, hipGetErrorString(he));
      break;
    }
    float* image = images[i % n_images];
    err = vy_render(scene, cuts[k], &cams[i], &ropts, image, ctxs[k], st);
    if (err == VY_OK && stats)
      err = render_frame_finish(cuts[k], ctxs[k], image, cams[i].width, cams[i].height, stats + i, st);
    if (err == VY_OK && frame_ms) {
      he = hipEventRecord(t1[i], st);
      if (he != hipSuccess) err = fail(VY_ERR_HIP, "vy_walkthrough: frame %lld: %s", (long long)i, hipGetErrorString(he));
    }
  }
  // the caller's stream continues after every slot, also after an error
  for (int k = 0; k < depth; ++k) {
    VY_HIP(hipEventRecord(joined[k], (hipStream_t)streams[k]));
    VY_HIP(hipStreamWaitEvent(caller, joined[k], 0));
  }
  if (err != VY_OK) return err;
  if (frame_ms) {
    VY_HIP(hipStreamSynchronize(caller));
    for (int64_t i = 0; i < n_frames; ++i) VY_HIP(hipEventElapsedTime(&frame_ms[i], t0[i], t1[i]));
  }
  return VY_OK;
}
