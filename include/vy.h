/*
 * vy.h - C ABI of the Voyager MI355X per-frame hot path.
 *
 * The library renders a 3D Gaussian Splatting scene stored as a level-of-detail
 * (LoD) tree, following "Voyager: Real-Time City-Scale 3D Gaussian Splatting on
 * Resource-Constrained Devices" (arXiv 2506.02774):
 *
 *   vy_lod_cut  - Section 3.1 "Cut Finding" and Section 4.1: the LoD cut, by a
 *                 full top-down search or by the temporal-aware search of
 *                 Algorithm 1 seeded with the previous frame's cut;
 *   vy_render   - Section 3.1 "Culling & Projection", "Sorting" and
 *                 "Rasterization", optionally with the preemptive alpha-filtering
 *                 of Section 4.2 (Eq. 3 and Eq. 4 moved to culling/projection)
 *                 and the lookup-table exponential of Eq. 5;
 *   vy_render_batch - the frames of several viewers (scenes, cameras, image
 *                 sizes) rendered with one launch per stage, each image
 *                 bitwise the one vy_render gives alone;
 *   vy_render_noalloc - vy_render with its scratch in a static device array,
 *                 for callers that cannot allocate;
 *   vy_render_backward - gradients of a rendered image with respect to the
 *                 cut's Gaussians (the adjoint of vy_render);
 *   vy_scene_partition - the height-2 subtree partition of Section 4.1 ("LoD
 *                 Tree Partitioning"), which VY_CUT_CHUNKED traverses;
 *   vy_scene_update_gaussians - new Gaussian parameters over the same tree
 *                 (training);
 *   inspection, stage timing and vy_measure_peaks - for tests and rooflines.
 * vy_serve.h builds two runtimes on these calls: a multi-viewer server and a
 * walkthrough renderer that keeps several frames of one camera path in flight.
 *
 * Conventions
 *   - Every entry point returns VY_OK (0) or a negative VY_ERR_* code; the
 *     message of the last error on the calling thread is vy_last_error().
 *   - "device" pointers are HIP device memory (for example torch CUDA tensors
 *     on ROCm); "host" pointers are ordinary memory. The library never
 *     allocates device memory: every device buffer comes from the caller,
 *     sized by the matching *_workspace_bytes() query (alignment 256 bytes).
 *   - `stream` is a hipStream_t (NULL = the null stream). All vy_lod_cut and
 *     vy_render work is enqueued asynchronously on it; only the functions that
 *     say so synchronise the stream.
 *   - Handles (vy_scene, vy_cut, vy_render_ctx) are host objects created by the
 *     library and released with their *_free(); they reference, but do not own,
 *     the caller's device buffers, which must outlive them. Calls that use one
 *     vy_cut or vy_render_ctx must not overlap; distinct handles may be used
 *     concurrently on distinct streams.
 *   - Camera: x_cam = R (x_world - pos), OpenCV axes (+x right, +y down,
 *     +z forward); pixel (i, j) is sampled at (i + 0.5, j + 0.5); pixel
 *     coordinates u = fx x/z + cx, v = fy y/z + cy.
 */
#ifndef VY_H
#define VY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  VY_OK = 0,
  VY_ERR_ARG = -1,      /* invalid argument (NULL handle, bad size, mismatched scene) */
  VY_ERR_HIP = -2,      /* a HIP runtime call failed */
  VY_ERR_CAPACITY = -3, /* a buffer was too small for this frame (output incomplete) */
  VY_ERR_STATE = -4,    /* handle used in an invalid state (e.g. empty previous cut) */
  VY_ERR_DEVICE = -5    /* a device-side consistency check failed */
};

const char* vy_last_error(void);
const char* vy_version(void);

/* Camera. R is row-major; rows are the camera's x (right), y (down) and
 * z (forward) axes in world coordinates. `pos` is the camera centre. */
typedef struct vy_camera {
  float R[9];
  float pos[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  float znear; /* near plane (0.2 m in the reference workloads) */
} vy_camera;

/* ------------------------------------------------------------------------ */
/* Scene                                                                     */
/* ------------------------------------------------------------------------ */

/* LoD tree (Section 3.1 "LoD Tree"): each node holds one Gaussian and a
 * contiguous range of children [first_child, first_child + child_count).
 * All arrays are DEVICE pointers, node-major, length n_nodes. Node 0 is the
 * root (parent -1); leaves have first_child = -1, child_count = 0.
 * Requirement (checked by vy_scene_validate): AABB(child) is contained in
 * AABB(parent) in float32, which makes the cut predicate monotone. */
typedef struct vy_scene_desc {
  int64_t n_nodes;
  const int32_t* parent;      /* [n] */
  const int32_t* first_child; /* [n] */
  const int32_t* child_count; /* [n] */
  const float* aabb_lo;       /* [n][3] */
  const float* aabb_hi;       /* [n][3] */
  const float* mean;          /* [n][3] */
  const float* log_scale;     /* [n][3] natural log of the per-axis std-dev */
  const float* quat;          /* [n][4] rotation (w, x, y, z), any norm > 0 */
  const float* opacity_logit; /* [n]    theta = sigmoid(logit) */
  const float* sh;            /* [n][16][3] SH degree-3 coefficients, index l*l+l+m;
                                 BORROWED: must stay valid while the scene lives */
} vy_scene_desc;

typedef struct vy_scene vy_scene;

/* Bytes of device workspace vy_scene_upload needs for n_nodes nodes. */
size_t vy_scene_workspace_bytes(int64_t n_nodes);

/* Packs the node arrays into the library's device layout in `workspace`
 * (caller-owned, >= vy_scene_workspace_bytes) and precomputes theta and
 * log(theta) per Gaussian (Section 4.2: log theta is computed once and stored),
 * and measures the tree depth (which sets the number of traversal launches).
 * Runs on `stream` and synchronises it; afterwards the desc arrays other than
 * `sh` may be released. Errors: VY_ERR_ARG for NULL pointers, n_nodes < 1, a
 * short workspace, or parent links that do not form a tree of depth < 1024;
 * VY_ERR_HIP on a HIP failure. */
int vy_scene_upload(const vy_scene_desc* desc, void* workspace, size_t workspace_bytes, void* stream,
                    vy_scene** out);

/* Device-side structural check (synchronises `stream`): counts nodes whose
 * parent/child links disagree or whose AABB is not inside the parent's.
 * Returns VY_OK with *n_bad = 0 for a valid tree. */
int vy_scene_validate(const vy_scene* scene, int64_t* n_bad, void* stream);

/* Replaces the Gaussians' parameters of an uploaded scene, keeping its tree
 * (links, AABBs, depth): repacks means, log-scales, quaternions and opacity
 * logits (theta and log theta recomputed, as at upload) from DEVICE arrays
 * laid out as in vy_scene_desc, and borrows `sh` in place of the previous SH
 * array. For training over a fixed tree (the backward pass of Section 3.1's
 * rendering): cuts of the scene stay valid, since the cut depends on the
 * AABBs only. A vy_render_backward of a frame rendered before the update is
 * refused (VY_ERR_STATE). Enqueued on `stream` (no synchronisation); the
 * arrays other than `sh` may be reused once it has run. VY_ERR_ARG for NULL
 * arguments. */
int vy_scene_update_gaussians(vy_scene* scene, const float* mean, const float* log_scale, const float* quat,
                              const float* opacity_logit, const float* sh, void* stream);
int64_t vy_scene_num_nodes(const vy_scene* scene);
int vy_scene_free(vy_scene* scene);

/* ------------------------------------------------------------------------ */
/* LoD cut (Section 3.1 "Cut Finding"; Section 4.1, Algorithm 1)             */
/* ------------------------------------------------------------------------ */

/* A cut handle holds, on the device, the frontier F (every non-expanded node
 * whose ancestors all expand, including nodes outside the view frustum) and
 * the cut C = F restricted to visible nodes, both as ascending int32 node ids.
 * F is the state the temporal search starts from in the next frame. */
typedef struct vy_cut vy_cut;

size_t vy_cut_workspace_bytes(int64_t n_nodes);
int vy_cut_create(const vy_scene* scene, void* workspace, size_t workspace_bytes, vy_cut** out);
int vy_cut_free(vy_cut* cut);

enum {
  VY_CUT_FRONTIER = 0, /* full search: top-down traversal from the root that visits
                          only expanded nodes and their children (Section 4.1,
                          "Fully-Streaming LoD Tree Traversal") */
  VY_CUT_FLAT = 1,     /* full search: exhaustive test of every node (the baseline
                          exhaustive search of Section 3.2 "Cut Finding") */
  VY_CUT_DFS = 2,      /* flag, for the top-down traversal of a full or temporal
                          search: each thread walks its queued node's subtree
                          depth first, 4 levels per launch, instead of the
                          default workgroup-wide breadth-first walk of 13 levels
                          per launch (frontier in LDS). The cut is the same
                          either way. */
  VY_CUT_CHUNKED = 4   /* flag: the traversal of Section 4.1 over the scene's
                          subtree partition (vy_scene_partition): a full search
                          streams chunks of height-2 subtrees in BFS order
                          through LDS on persistent workgroups that take the
                          chunks from an atomic queue; a temporal search runs
                          Algorithm 1 per subtree (TOP: the parent subtree is
                          searched, BOTTOM: the child subtrees). The cut is the
                          same. Searches of one scene in this mode share the
                          partition's per-subtree stamps and must not overlap.
                          Not with VY_CUT_FLAT or VY_CUT_DFS. */
};

/* Subtree partition of a scene's tree for VY_CUT_CHUNKED (Section 4.1, "LoD
 * Tree Partitioning"): the tree is split into subtrees of height 2 (a root at
 * depth 0, 3, 6, ... with its children and grandchildren), ordered by root id
 * (BFS order for a breadth-first numbering), their nodes stored subtree after
 * subtree (32 bytes per node), and packed greedily into chunks of consecutive
 * subtrees of at most 2048 nodes (64 KB of LDS), which for contiguous chunks
 * gives the fewest chunks, the optimum of the paper's packing problem (Eq. 1
 * and 2). Built on the host from the uploaded scene (copied back), then copied
 * into `workspace` (DEVICE, caller-owned, >= vy_scene_partition_bytes(n_nodes)
 * bytes) and attached to the scene until vy_scene_free or the next call.
 * Synchronises `stream`. Errors: VY_ERR_ARG for a short workspace, a tree whose
 * parents are not numbered before their children, a subtree of more than 64
 * nodes (fanout above 7) or a node with more than 2047 children. */
size_t vy_scene_partition_bytes(int64_t n_nodes);
int vy_scene_partition(vy_scene* scene, void* workspace, size_t workspace_bytes, void* stream);

/* The host half of vy_scene_partition, exposed for checking without a GPU:
 * from HOST arrays parent, first_child, child_count [n] it writes sub_of [n]
 * (each node's subtree), local [n] (each node's position in the subtree-major
 * order), sub_root [n] and sub_rec [n + 1] (each subtree's root and first
 * position; *n_sub subtrees) and chunk_sub [n + 1] (each chunk's first
 * subtree; *n_chunks chunks). Errors as vy_scene_partition. */
int vy_partition_plan(int64_t n, const int32_t* parent, const int32_t* first_child, const int32_t* child_count,
                      int32_t* sub_of, int32_t* local, int64_t* n_sub, int32_t* sub_root, int32_t* sub_rec,
                      int32_t* chunk_sub, int64_t* n_chunks);

/* Computes the cut for `cam` at LoD granularity `tau` (pixels).
 * Predicate (Section 3.1): node n expands iff it has children, its AABB is not
 * outside the view frustum (4 side planes through the camera centre and the
 * near plane), and fx * ext(n) > tau * dist(n), where ext is the longest AABB
 * side and dist the distance from the camera centre to the AABB.
 *   prev == NULL : full search, method `full_mode` (VY_CUT_FRONTIER or
 *                  VY_CUT_FLAT, optionally | VY_CUT_DFS).
 *   prev != NULL : temporal search (Algorithm 1) seeded with prev's frontier;
 *                  prev must hold a cut of the same scene (VY_ERR_STATE if it
 *                  has never been computed, VY_ERR_ARG for another scene).
 *                  prev == out is allowed. The result is identical, bit for
 *                  bit, to the full search. `full_mode` may carry
 *                  VY_CUT_DFS here too.
 * Enqueued on `stream`. */
int vy_lod_cut(const vy_scene* scene, const vy_camera* cam, float tau, vy_cut* prev, vy_cut* out,
               int full_mode, void* stream);

/* Synchronises `stream`; returns |F| and |C| of the last computed cut, and
 * VY_ERR_DEVICE if a device-side bound was hit while computing it. */
int vy_cut_counts(const vy_cut* cut, int64_t* n_frontier, int64_t* n_cut, void* stream);

/* Device pointers to the ascending id arrays of the last computed cut (valid
 * until the next vy_lod_cut writing this handle) and to the device int32
 * counters {|F|, |C|}. Any pointer argument may be NULL. */
int vy_cut_arrays(const vy_cut* cut, const int32_t** frontier, const int32_t** cut_ids,
                  const int32_t** counts);

/* Replace the frontier of `cut` with `n` caller-given node ids (device,
 * ascending, forming a valid frontier: one node on every root-to-leaf path),
 * e.g. to seed the temporal search from an arbitrary state. Enqueued. */
int vy_cut_set_frontier(vy_cut* cut, const int32_t* ids, int64_t n, void* stream);

/* ------------------------------------------------------------------------ */
/* Rendering (Section 3.1 Culling & Projection, Sorting, Rasterization;     */
/* Section 4.2 preemptive alpha-filtering)                                   */
/* ------------------------------------------------------------------------ */

typedef struct vy_render_opts {
  int32_t alpha_filter; /* 0: plain pipeline. 1: preemptive alpha-filtering
                           (Eq. 4 applied per Gaussian, per Gaussian-tile pair at
                           binning and per pixel before the exponential). The
                           image is bitwise identical either way. */
  float bg[3];          /* background colour (default black) */
  int32_t save_state;   /* 1: also write the per-pixel final transmittance and
                           contributor count (needed by the backward pass) */
  int32_t split_min_pairs; /* > 0: tiles with more pairs are blended by several
                              workgroups over depth bins, then composited (0: no
                              splitting). The image is bitwise the same for any
                              value; splitting forgoes early termination. */
  int32_t walk;         /* how a band of 16x4 pixels walks its tile list: 0 (auto)
                           each pixel over its own entries, and once at most 4
                           pixels of the band still blend, a chunk's entries in
                           parallel for one pixel at a time; tiles with more
                           than 4096 pairs are blended band by band by waves of
                           their own (band_jobs); 1: all pixels together over
                           every entry; 2: each pixel over its own entries (1
                           and 2 blend every tile with one workgroup). The
                           image is bitwise the same for any value. */
  int32_t lut_entries;  /* 0: alpha uses the exponential. m in 1..128: the
                           lookup table of Section 4.2 (Eq. 5): e^rho is read
                           from m + 1 values e^(-5.55 k / m), k = 0..m, at
                           k = round(rho / -5.55 * m) (clamped to m), held in
                           LDS. An approximation: the image differs from the
                           exact one (filtered and unfiltered still agree bit
                           for bit: the preemptive check keeps a margin of half
                           an interval more). Not with split_min_pairs > 0. */
  int32_t band_jobs;    /* with walk = 0, how the tiles of more than 4096 pairs
                           are cut into wave jobs: 1 (latency) halves of 16x4
                           bands on more dedicated workgroups, the shortest
                           frame when frames run one at a time; 2 (throughput)
                           whole bands on fewer workgroups, less work in all,
                           faster when frames overlap; 0 (default) 1 for
                           vy_render, 2 for vy_render_batch, and in
                           vy_serve.h 2 when frames overlap (vy_walkthrough
                           with depth > 1, a server with several frames in
                           flight). The image is bitwise the same for any
                           value; other values are refused (VY_ERR_ARG). */
} vy_render_opts;

typedef struct vy_render_ctx vy_render_ctx;

/* Workspace for rendering cuts of at most max_gaussians nodes into images of
 * at most max_width x max_height with at most max_pairs Gaussian-tile pairs. */
size_t vy_render_workspace_bytes(int64_t max_gaussians, int32_t max_width, int32_t max_height,
                                 int64_t max_pairs);
int vy_render_ctx_create(int64_t max_gaussians, int32_t max_width, int32_t max_height, int64_t max_pairs,
                         void* workspace, size_t workspace_bytes, vy_render_ctx** out);
int vy_render_ctx_free(vy_render_ctx* ctx);

/* Renders the cut C of `cut` seen from `cam` into `image` (DEVICE, float32,
 * planar [3][height][width], caller-owned). Stages: EWA projection with SH
 * colour; 16x16-tile binning (with the pair-level alpha filter when enabled);
 * a stable radix sort by (tile, depth) with depth ties in node-id order;
 * per-tile front-to-back blending with alpha = min(0.99, theta e^rho) (Eq. 3),
 * skipping alpha < 1/255 and stopping before T falls below 1e-4.
 * Enqueued on `stream`. VY_ERR_ARG if the camera exceeds the context's image
 * size or the cut belongs to another scene. A pair overflow is reported by
 * vy_render_status (the image is then incomplete). */
int vy_render(const vy_scene* scene, const vy_cut* cut, const vy_camera* cam, const vy_render_opts* opts,
              float* image, vy_render_ctx* ctx, void* stream);

/* Rendering without allocation, for callers that cannot allocate device
 * memory or create a context (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc). The same stages and kernels as
 * vy_render, so the image is bitwise the one vy_render writes; the context's
 * scratch (projected Gaussians, sort buffers, counters, look-back words,
 * per-pixel state) is instead a static device array of
 * VY_NOALLOC_SCRATCH_BYTES that each GPU holds from the first call on it until
 * the process ends, laid out at fixed capacities: a cut of at most
 * VY_NOALLOC_MAX_GAUSSIANS entries, VY_NOALLOC_MAX_PAIRS Gaussian-tile pairs,
 * images of at most VY_NOALLOC_MAX_WIDTH x VY_NOALLOC_MAX_HEIGHT. It calls no
 * hipMalloc/hipFree and allocates no host memory; the first call on a device
 * looks up the array's address and clears its look-back words with a kernel on
 * `stream`.
 *   image  : DEVICE float32 [3][height][width], caller-owned (written).
 *   counts : DEVICE uint32[4], caller-owned, or NULL; receives {pairs needed,
 *            Gaussians with at least one pair, the cut size if it exceeds
 *            VY_NOALLOC_MAX_GAUSSIANS (else 0), device-side bound hits}. A
 *            frame whose pairs exceed VY_NOALLOC_MAX_PAIRS, or whose cut
 *            exceeds VY_NOALLOC_MAX_GAUSSIANS, is rendered incomplete: the
 *            caller checks counts[0] and counts[2].
 * Errors: VY_ERR_ARG for an image larger than the maximum, save_state or
 * split_min_pairs (they need a context), or the arguments vy_render refuses;
 * VY_ERR_HIP if the array's address cannot be obtained.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (on concurrent streams or host
 * threads) race and must be serialised by the caller. Enqueued on `stream`. */
#define VY_NOALLOC_SCRATCH_BYTES (64u << 20)
#define VY_NOALLOC_MAX_GAUSSIANS (1 << 18)
#define VY_NOALLOC_MAX_PAIRS (1 << 20)
#define VY_NOALLOC_MAX_WIDTH 1280
#define VY_NOALLOC_MAX_HEIGHT 720
int vy_render_noalloc(const vy_scene* scene, const vy_cut* cut, const vy_camera* cam, const vy_render_opts* opts,
                      float* image, uint32_t* counts, void* stream);

/* ------------------------------------------------------------------------ */
/* Batched rendering: the frames of several viewers in one launch per stage  */
/* ------------------------------------------------------------------------ */

/* One viewer's frame in a batch: its scene, its computed cut, its camera and
 * its image (DEVICE float32 [3][height][width], caller-owned). */
typedef struct vy_view {
  const vy_scene* scene;
  const vy_cut* cut;
  vy_camera cam;
  float* image;
} vy_view;

typedef struct vy_batch_ctx vy_batch_ctx;

#define VY_BATCH_MAX_VIEWS 64
#define VY_BATCH_MAX_TILES 65536

/* Workspace for batches of at most max_views views whose cuts hold at most
 * max_gaussians Gaussians in all, with at most max_tiles 16x16 tiles in all
 * (<= VY_BATCH_MAX_TILES, e.g. 8 views at 1920x1080) and max_pairs pairs.
 * 0 for invalid arguments. */
size_t vy_batch_workspace_bytes(int32_t max_views, int64_t max_gaussians, int64_t max_tiles, int64_t max_pairs);
/* Also allocates a small ring of pinned HOST buffers (and events) for the
 * batch descriptor, released by vy_batch_ctx_free; synchronises the device. */
int vy_batch_ctx_create(int32_t max_views, int64_t max_gaussians, int64_t max_tiles, int64_t max_pairs,
                        void* workspace, size_t workspace_bytes, vy_batch_ctx** out);
int vy_batch_ctx_free(vy_batch_ctx* ctx);

/* Renders n_views frames (Section 3.1 "Culling & Projection", "Sorting",
 * "Rasterization"; Section 4.2 with opts->alpha_filter) with one launch per
 * stage for the whole batch: the views' cuts are concatenated, projected with
 * each view's own scene and camera, sorted by depth together, and their pairs
 * keyed by global tile (view v owns the tiles after those of views 0..v-1, so
 * the view is the key's top part) and sorted by tile; each tile is blended
 * into its view's image. Every image is bitwise the one vy_render writes for
 * that view alone with the same options. opts->save_state and
 * split_min_pairs must be 0. The descriptor is copied on `stream` (a pinned
 * ring of 4 slots: a call waits for the copy of the call 4 before it).
 * Enqueued on `stream`; calls on one batch context must not overlap. Errors:
 * VY_ERR_ARG for a bad view, more views or tiles than the context holds;
 * VY_ERR_STATE for a cut never computed. Overflows of max_gaussians or
 * max_pairs are reported by vy_batch_status (the images are then incomplete). */
int vy_render_batch(const vy_view* views, int32_t n_views, const vy_render_opts* opts, vy_batch_ctx* ctx,
                    void* stream);

/* As vy_render_status, for the last batch: the batch's pairs and Gaussians
 * with pairs, VY_ERR_CAPACITY when they exceeded the context. Synchronises
 * `stream`. */
int vy_batch_status(vy_batch_ctx* ctx, int64_t* n_pairs, int64_t* n_visible, void* stream);

/* Synchronises `stream`; returns the last frame's pair count and number of
 * projected (non-culled) Gaussians, VY_ERR_CAPACITY if the pairs exceeded
 * max_pairs (then *n_pairs is the number required), VY_ERR_DEVICE if a
 * device-side wait bound was hit. */
int vy_render_status(vy_render_ctx* ctx, int64_t* n_pairs, int64_t* n_visible, void* stream);

/* Device pointers into the context's saved state of the last frame (written
 * only with save_state = 1), each [H][W]: final transmittance, number of
 * blended Gaussians, the number of tile-list entries the pixel evaluated
 * before blending stopped (its tile's whole list if it never stopped; -1 for
 * pixels of tiles blended in split mode), and the position in the sorted pair
 * list of the last Gaussian the pixel blended (-1 if none; not written in
 * split mode); and the projected Gaussians' 2D means [n][4] (cut order, first
 * two floats). Any argument may be NULL. */
int vy_render_saved(const vy_render_ctx* ctx, const float** T_final, const int32_t** n_contrib,
                    const int32_t** n_eval, const int32_t** last_contrib, const float** mean2d);

/* Device pointers to the last frame's sorted pairs ([n_pairs] each): the tile
 * key (tile id in bits 0..15; above it the pair's pixel box within the tile,
 * 4 bits each: first and last column, first and last row that may hold a
 * pixel centre the Gaussian reaches) and the cut position of the Gaussian;
 * and the tile ranges ([tiles] uint2, begin and end in the pair list). */
int vy_render_pairs(const vy_render_ctx* ctx, const uint32_t** tile_keys, const uint32_t** cut_pos,
                    const uint32_t** ranges);
/* Device pointers to the projected records of the cut ([n] float4 each, cut
 * order: mean2d and rho coefficients A, B; C, theta, filter threshold,
 * depth; rgb and the packed pixel half-extents) and the binning records
 * ([n] uint4: tile rect x0 | y0 << 16, x1 | y1 << 16, kept-tile mask, and the
 * pair count; for rects of at most 32 tiles (mask != 0) the count is the low
 * 8 bits and the pixel box of vy_render_pairs' keys, for the rect's first and
 * last tiles, the 16 bits above it). */
int vy_render_projected(const vy_render_ctx* ctx, const float** rec0, const float** rec1, const float** rec2,
                        const uint32_t** bin_rec);

/* ------------------------------------------------------------------------ */
/* Backward pass: gradients of a rendered image                             */
/* ------------------------------------------------------------------------ */

/* Gradient outputs: DEVICE float32 arrays indexed by node id, laid out like the
 * arrays given to vy_scene_upload. Every Gaussian of the cut writes its own
 * rows (zeros where it did not reach the image); rows of other nodes are not
 * touched. Any output pointer may be NULL (not written). */
typedef struct vy_grads {
  float* mean;            /* [n][3] world-space means */
  float* log_scale;       /* [n][3] */
  float* quat;            /* [n][4] (w, x, y, z) */
  float* opacity_logit;   /* [n] */
  float* sh;              /* [n][48] (16 coefficients x 3 channels) */
  float* mean2d;          /* [n][2] screen-space means (a by-product) */
  const float* quat_raw;  /* [n][4] DEVICE: the quaternions as given to
                             vy_scene_upload, which normalises them; `quat` is
                             then the gradient for these raw values. NULL: for
                             the unit quaternion. */
} vy_grads;

/* dL/d(parameters) of the image of the last vy_render on `ctx`, given
 * dL/dimage (DEVICE float32, planar [3][H][W]). That render must have used
 * save_state = 1, no split tiles and the exact exponential, with this scene,
 * this cut (not recomputed since) and this camera (VY_ERR_STATE otherwise).
 * The depth order, the pixel boxes and the alpha* / transmittance decisions of
 * that frame are held fixed (piecewise differentiation).
 * Steps:
 *   1. The blend (Section 3.1 "Rasterization", Eq. 3) is replayed back to
 *      front from each pixel's last blended Gaussian, recovering the
 *      transmittance from the saved final value.
 *   2. Per Gaussian, the gradients of its 2D mean, conic, opacity and colour
 *      are summed over each wave and added with atomics.
 *   3. The projection (Section 3.1 "Culling & Projection": EWA with the
 *      Jacobian clamps and the low-pass), the SH colour with its clamp, the
 *      scale exponential, the quaternion rotation and the opacity sigmoid are
 *      differentiated per Gaussian.
 * Overwrites the depth-sort and binning intermediates of the context (see
 * vy_render_projected). Enqueued on `stream`. */
int vy_render_backward(const vy_scene* scene, const vy_cut* cut, const vy_camera* cam, const float* dL_dimage,
                       const vy_grads* grads, vy_render_ctx* ctx, void* stream);

/* ------------------------------------------------------------------------ */
/* Stage timing (HIP events recorded around every kernel launch)            */
/* ------------------------------------------------------------------------ */

enum {
  VY_STAGE_LOD_SETUP = 0,
  VY_STAGE_LOD_FLAT,
  VY_STAGE_LOD_CLASSIFY,
  VY_STAGE_LOD_TRAVERSE,
  VY_STAGE_LOD_COMPACT,
  VY_STAGE_RENDER_SETUP,
  VY_STAGE_PROJECT,
  VY_STAGE_DEPTH_SORT,
  VY_STAGE_PAIR_SCAN,
  VY_STAGE_EMIT,
  VY_STAGE_TILE_SORT,
  VY_STAGE_RANGES,
  VY_STAGE_BLEND_PLAN,
  VY_STAGE_BLEND,
  VY_STAGE_BWD_BLEND,    /* vy_render_backward: blend replay */
  VY_STAGE_BWD_PROJECT,  /* vy_render_backward: projection, SH, sigmoid */
  VY_NUM_STAGES
};

/* Starts recording (capacity = max number of launches to record). While
 * recording, each launch by this thread is bracketed by HIP events on its
 * stream. */
int vy_profile_begin(int64_t capacity);
/* Stops recording, synchronises the recorded events and writes the summed
 * milliseconds and launch counts per stage (arrays of VY_NUM_STAGES). */
int vy_profile_end(double* stage_ms, int64_t* stage_launches);
const char* vy_stage_name(int stage);

/* Practical vector peaks of the current device, for the rooflines: probe
 * kernels time FP32 fused multiply-adds (8 independent chains per lane,
 * compiled like every kernel of the library, i.e. without packed FP32
 * instructions) and the hardware exponential (v_exp_f32). Writes TFLOP/s
 * (2 per FMA) and G exponentials/s. scratch: device, at least
 * vy_measure_peaks_bytes() bytes (overwritten). Runs on `stream` and
 * synchronises it. VY_ERR_ARG for a NULL or short argument. */
size_t vy_measure_peaks_bytes(void);
int vy_measure_peaks(float* scratch, size_t scratch_bytes, double* fma_tflops, double* exp_gops, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* VY_H */
