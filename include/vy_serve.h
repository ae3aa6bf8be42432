/*
 * vy_serve.h - C ABI of the runtimes built on vy.h: the multi-viewer serving
 * runtime, and the walkthrough renderer that keeps several frames of one
 * viewer's camera path in flight.
 *
 * Many viewers, each walking through one of several resident scenes at its
 * own resolution, ask for frames at their own times. The runtime
 *   - keeps every admitted viewer's state resident in device memory between
 *     its frames: the LoD frontier of its previous frame, which the
 *     temporal-aware search of Algorithm 1 (Section 4.1) starts from, and the
 *     projection, sort and blend buffers of vy_render;
 *   - admits a viewer when a viewer slot and enough device memory are free
 *     (first come, first served) and releases both after its last frame;
 *   - issues frames on several HIP streams, so that frames of different
 *     viewers run on the GPU at the same time.
 * Every frame is exactly the per-frame path of vy.h: vy_lod_cut (a full
 * search for a viewer's first frame, Algorithm 1 afterwards) then vy_render
 * (Section 3.1 with the alpha filter of Section 4.2 when asked), so a viewer's
 * images are bit for bit those it gets when rendered alone.
 *
 * Device memory: the runtime never allocates device memory. Per-viewer state
 * is carved out of one caller-owned device range by a vy_arena. Host-side
 * bookkeeping lives in the handles. Conventions (status codes, streams,
 * vy_last_error) are those of vy.h.
 */
#ifndef VY_SERVE_H
#define VY_SERVE_H

#include "vy.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------------ */
/* Device memory arena                                                      */
/* ------------------------------------------------------------------------ */

/* Host-side bookkeeping of the caller's device range [base, base + bytes):
 * first fit over the free blocks in address order, sizes rounded up to
 * 256-byte granules, neighbouring free blocks merged on release. The arena
 * never reads or writes the range itself (these calls work without a GPU).
 * base must be 256-byte aligned and stay allocated while the arena is used. */
typedef struct vy_arena vy_arena;

int vy_arena_create(void* base, size_t bytes, vy_arena** out);
int vy_arena_free(vy_arena* arena);
/* *out = start of a block of at least `bytes` (> 0); VY_ERR_CAPACITY (and
 * *out = NULL) when no free block is large enough. */
int vy_arena_alloc(vy_arena* arena, size_t bytes, void** out);
/* Returns a block to the arena; VY_ERR_ARG unless `ptr` starts a live block. */
int vy_arena_release(vy_arena* arena, void* ptr);
/* Bytes in live blocks, size of the largest free block, number of live
 * blocks and of free blocks. Any pointer may be NULL. */
int vy_arena_stats(const vy_arena* arena, size_t* used, size_t* largest_free, int64_t* n_live,
                   int64_t* n_free_blocks);

/* ------------------------------------------------------------------------ */
/* Viewer sessions and frame requests                                       */
/* ------------------------------------------------------------------------ */

/* One viewer session: the scene it walks through and how it is rendered. */
typedef struct vy_session {
  const vy_scene* scene;
  int32_t width, height;   /* image size of every frame of the session */
  float tau;               /* LoD granularity in pixels (vy_lod_cut) */
  int32_t alpha_filter;    /* vy_render_opts.alpha_filter */
  int64_t max_gaussians;   /* cut capacity of its render context; 0: chosen by
                              the runtime (see below) */
  int64_t max_pairs;       /* pair capacity; 0: chosen by the runtime */
} vy_session;

/* Capacities left to the runtime start at min(scene nodes, 2 * width *
 * height) Gaussians and 4 * width * height pairs (the cut's size depends on
 * the scene and tau more than on the image size, the pairs' on the cut), and
 * grow when a frame overflows them: the session pauses until its unfinished
 * frames are done, its render workspace is replaced by one with twice the
 * capacity, or 1.25 times what the frame needed if that is more, and the
 * overflowed frames are rendered again. Capacities the caller sets are kept;
 * frames that overflow them are reported in their flags. */

/* Device bytes one session holds when it is admitted (its vy_cut workspace,
 * one image and its initial render workspace), 0 for an invalid description. */
size_t vy_session_bytes(const vy_session* session);

/* One frame asked for by a session. */
typedef struct vy_frame_req {
  int32_t session;    /* index into the sessions array */
  int32_t reserved;   /* 0 */
  double t_arrival;   /* seconds after the start of the run; non-decreasing
                         over the request array */
  vy_camera cam;      /* width and height equal to the session's */
  float* image;       /* device [3][height][width] output, or NULL for the
                         session's own buffer (overwritten by its next frame) */
} vy_frame_req;

/* Device record written by the last kernel of every frame (for a batched
 * frame, n_pairs, n_visible and flags 1, 2, 4 are those of its batch). */
typedef struct vy_frame_stats {
  uint64_t image_hash;  /* sum over flat index i of the image of
                           mix64((i << 32) | bits of image[i]) modulo 2^64,
                           mix64 = the SplitMix64 finaliser: changes whenever
                           any value of the image changes */
  uint32_t n_cut;       /* |C| */
  uint32_t n_pairs;     /* Gaussian-tile pairs the frame needed */
  uint32_t n_visible;   /* projected Gaussians with at least one pair */
  uint32_t flags;       /* 1: pairs exceeded max_pairs; 2: the cut exceeded
                           max_gaussians; 4: a device-side wait bound was hit in
                           vy_render; 8: in vy_lod_cut. Any flag: image incomplete */
  uint32_t n_frontier;  /* |F| */
  uint32_t reserved;
} vy_frame_stats;

/* Host record of every frame, times in seconds after the start of the run. */
typedef struct vy_frame_result {
  double t_admit;     /* its session became resident */
  double t_dispatch;  /* the host enqueued the frame */
  double t_start;     /* the GPU reached the frame on its stream (HIP event) */
  double t_done;      /* the frame's last kernel ended (HIP event) */
  int32_t status;     /* VY_OK, or the error of enqueueing the frame (its
                         times are then those of the attempt) */
  int32_t stream;     /* index of the stream it ran on */
} vy_frame_result;

/* ------------------------------------------------------------------------ */
/* Server                                                                   */
/* ------------------------------------------------------------------------ */

typedef struct vy_server_config {
  vy_arena* arena;        /* device memory for resident sessions (borrowed) */
  int32_t n_streams;      /* 1..16 */
  void* const* streams;   /* n_streams distinct hipStream_t (borrowed) */
  int32_t max_inflight;   /* frames enqueued and unfinished per stream, >= 1 */
  int32_t max_viewers;    /* sessions resident at once, >= 1 */
  int32_t max_batch;      /* 0 or 1: every frame is its own vy_render. 2..64:
                             frames dispatched to a stream in one scheduling
                             pass (one per session, same alpha_filter, at most
                             VY_BATCH_MAX_TILES tiles) are fused: their
                             vy_lod_cut calls, then one vy_render_batch over
                             them. Sessions then hold no render workspace:
                             each stream has one batch context, carved from the
                             arena for the duration of the run. */
  int32_t reserved;       /* 0 */
  int64_t batch_gaussians; /* capacities of each stream's batch context (cut
                              Gaussians and pairs of all its frames together);
                              frames of a batch that overflows them are
                              flagged (1 or 2), not rendered again */
  int64_t batch_pairs;
} vy_server_config;

typedef struct vy_server vy_server;

int vy_server_create(const vy_server_config* config, vy_server** out);
int vy_server_free(vy_server* server);

enum {
  VY_RUN_REALTIME = 1  /* release every request at its arrival time on the
                          host clock (otherwise all are available at once) */
};

/* Serves a trace of frame requests and returns when every frame is done.
 *   sessions[n_sessions]: the sessions the requests refer to. A session is
 *     admitted at its first request (first come, first served, when a viewer
 *     slot and vy_session_bytes() of arena are free; the first request of a
 *     session that can never fit fails with VY_ERR_CAPACITY before anything
 *     runs) and released after its last request has finished.
 *   reqs[n_reqs]: sorted by t_arrival; a session's frames are rendered in
 *     array order (each after the previous one of the same session has been
 *     enqueued, so the temporal search always starts from the previous frame).
 *   Scheduling: among admitted sessions with released frames, the oldest
 *     request goes first. A session with unfinished frames stays on its
 *     stream; an idle one takes the stream with the fewest unfinished frames.
 *   stats: device [n_reqs] (zeroed by the call), or NULL: the records are
 *     then kept in a block of the arena for the duration of the call.
 *   results: host [n_reqs]; a re-rendered frame reports its last attempt.
 *   A frame rendered again after its session grew may overwrite the
 *   session's own buffer after a later frame did; pass an image per request
 *   to keep every frame. The call uses n_reqs * 32 bytes of pinned host
 *   memory (hipHostMalloc) for the records' host copies.
 * Returns VY_OK when every frame was enqueued and finished (per-frame
 * problems are in results[i].status and stats[i].flags), VY_ERR_ARG for an
 * invalid trace (nothing runs), VY_ERR_HIP if a HIP call failed (the run is
 * abandoned after the streams are synchronised). Not thread-safe per server. */
int vy_server_run(vy_server* server, const vy_session* sessions, int32_t n_sessions, const vy_frame_req* reqs,
                  int64_t n_reqs, int32_t flags, vy_frame_stats* stats, vy_frame_result* results);

/* Counters of the last run: sessions admitted, sessions that had to wait for
 * admission, peak resident sessions, peak arena bytes in use, render
 * workspaces grown and frames rendered again. Any pointer may be NULL. */
int vy_server_last_run(const vy_server* server, int64_t* n_admitted, int64_t* n_waited, int64_t* peak_resident,
                       size_t* peak_bytes, int64_t* n_regrown, int64_t* n_redone);

/* The admission, scheduling and growth policy of vy_server_run, run against
 * a model of the GPU instead of the GPU (no HIP call; works without a GPU):
 * frame i keeps its stream busy for service_s[i] seconds from the later of
 * its dispatch and the end of the stream's previous frame, streams run
 * independently, time is virtual and dispatch takes none of it. Session s
 * holds session_bytes[s] (> 0) plus, when pair_capacity is given, a render
 * block of 16 bytes per pair of capacity, initially pair_capacity[s]; with
 * need_pairs[n_reqs] (requires pair_capacity) a frame overflows when it
 * needs more pairs than the capacity it was dispatched with, and the session
 * grows as in vy_server_run. `config->streams` is not used. Fills
 * results[n_reqs] as vy_server_run does (t_start, t_done in model time) and
 * counters[6] (may be NULL) with the values of vy_server_last_run. */
int vy_server_simulate(const vy_server_config* config, const int64_t* session_bytes, const int64_t* pair_capacity,
                       int32_t n_sessions, const vy_frame_req* reqs, int64_t n_reqs, const double* service_s,
                       const uint32_t* need_pairs, int32_t flags, vy_frame_result* results, int64_t* counters);

/* ------------------------------------------------------------------------ */
/* Walkthrough: one viewer's camera path with several frames in flight      */
/* ------------------------------------------------------------------------ */

enum {
  VY_WALK_FULL_EACH = 256  /* in vy_walkthrough's full_mode: every frame is a
                              full search (prev is not used), and the frames do
                              not wait for each other */
};

/* Renders frames i = 0..n_frames-1 of one camera path. Frame i is
 * vy_lod_cut(scene, cams[i], tau, from, cut_i, full_mode) with `from` =
 * frame i-1's cut (the temporal search of Algorithm 1, Section 4.1), or
 * `prev` for frame 0 (NULL: a full search), followed by
 * vy_render(scene, cut_i, cams[i], opts, images[i % n_images], ctx_i) (Section
 * 3.1, with Section 4.2 per opts). Every cut and image is therefore bit for bit
 * the one a loop over those two calls produces.
 * full_mode: as in vy_lod_cut for the full searches (VY_CUT_FRONTIER,
 * VY_CUT_FLAT, | VY_CUT_DFS), optionally | VY_WALK_FULL_EACH.
 * Up to `depth` frames are in flight. Frame i uses slot i % depth: the cut
 * cuts[slot], the context ctxs[slot], the stream streams[slot]. Its search
 * waits (a HIP event) only for frame i-1's search, so frame i's rendering
 * overlaps the searches and renderings of the next depth - 1 frames. With
 * depth = 1 the frames run one after the other on streams[0].
 *   cams: host [n_frames], each no larger than its slot's context.
 *   cuts, ctxs, streams: host arrays of `depth` (1..16) distinct handles /
 *     hipStream_t (borrowed; one stream may be NULL, the null stream). prev
 *     may be one of cuts. After the call the
 *     last frame's cut is in cuts[(n_frames - 1) % depth].
 *   images: host array of n_images device images [3][H][W] (caller-owned);
 *     n_images must be a positive multiple of depth, so that an image is only
 *     written by one slot.
 *   stats: device [n_frames] or NULL: zeroed, then frame i's record as in
 *     vy_server_run (image hash, |C|, pairs, flags: a capacity or wait bound
 *     hit by any frame shows there, whereas vy_render_status of a context only
 *     reports the last frame it rendered).
 *   frame_ms: host [n_frames] or NULL: GPU time of each frame from the start
 *     of its search to the end of its rendering (HIP timing events on its
 *     stream); the call then synchronises `stream` and fills it before
 *     returning VY_OK (it is left as is when the call fails).
 *   stream: the caller's stream; it may also be one of streams. The frames
 *     start after the work already enqueued on it, and work enqueued on it
 *     after the call starts after every frame. (HIP maps a process's streams
 *     onto a few hardware queues, 4 by default, and streams beyond that share
 *     a queue, where their frames no longer overlap: keep the distinct
 *     streams among `streams` and `stream` within the queue count, for
 *     example by passing `stream` as streams[0].)
 * Returns VY_ERR_ARG for invalid arguments (nothing is enqueued). An error of
 * vy_lod_cut or vy_render for frame i (argument checks, HIP) stops the call
 * there and is returned; frames before i still complete, `stream` still
 * waits for them, and the records of frames from i on stay zero. Not
 * thread-safe with respect to the handles it uses. */
int vy_walkthrough(const vy_scene* scene, const vy_camera* cams, int64_t n_frames, float tau, int32_t full_mode,
                   const vy_render_opts* opts, vy_cut* prev, int32_t depth, vy_cut* const* cuts,
                   vy_render_ctx* const* ctxs, void* const* streams, float* const* images, int64_t n_images,
                   vy_frame_stats* stats, float* frame_ms, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* VY_SERVE_H */
