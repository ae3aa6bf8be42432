// Shared internals of the Voyager HIP library (gfx950): handle layouts, error
// reporting, launch timing and wave64 device primitives.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/vy.h"

namespace vy {

// ---------------------------------------------------------------- errors ----

void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);

#define VY_HIP(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return ::vy::fail(VY_ERR_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),    \
                        __FILE__, __LINE__);                                                  \
  } while (0)

#define VY_LAUNCHED()                                                                         \
  do {                                                                                        \
    hipError_t e_ = hipGetLastError();                                                        \
    if (e_ != hipSuccess)                                                                     \
      return ::vy::fail(VY_ERR_HIP, "kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                  \
  } while (0)

// ---------------------------------------------------------------- timing ----

// Brackets a launch with HIP events when vy_profile_begin() is active.
void prof_mark(int stage, hipStream_t s, bool end);
struct ProfScope {
  int stage;
  hipStream_t s;
  ProfScope(int st, hipStream_t str) : stage(st), s(str) { prof_mark(stage, s, false); }
  ~ProfScope() { prof_mark(stage, s, true); }
};

// ------------------------------------------------------------- workspace ----

struct Carver {
  uintptr_t base, cur, end;
  explicit Carver(void* p, size_t bytes) : base((uintptr_t)p), cur((uintptr_t)p), end((uintptr_t)p + bytes) {}
  template <class T>
  T* take(size_t count) {
    cur = (cur + 255) & ~uintptr_t(255);
    T* r = reinterpret_cast<T*>(cur);
    cur += count * sizeof(T);
    return r;
  }
  size_t used() const { return cur - base; }
  bool ok() const { return cur <= end; }
};

// ----------------------------------------------------------------- handles ----

constexpr uint32_t kSceneMagic = 0x56595343u, kCutMagic = 0x56594355u, kCtxMagic = 0x56595243u;

struct Scene {
  uint32_t magic;
  int64_t n;
  // LoD record: {lo.x, lo.y, lo.z, first_child}, {hi.x, hi.y, hi.z, parent} (ints stored as bits)
  float4* lod;
  int32_t* ccount;   // child counts
  // Gaussian record: {mean.xyz, log theta}, {scale.xyz, theta}, {unit quaternion w,x,y,z}
  float4* gauss;
  const float* sh;   // borrowed [n][48]
  int levels;        // tree depth + 1 (computed at upload)
  int32_t* scratch;  // small device scratch for validate
  uint64_t params_version;  // bumped by each vy_scene_update_gaussians
  struct Partition* part;   // subtree partition (vy_scene_partition), or null
};

// Height-2 subtrees of the LoD tree (a root at depth 0, 3, 6, ... with its
// children and grandchildren) in BFS order of their roots, their nodes stored
// subtree after subtree, and chunks of consecutive subtrees of at most
// kChunkNodes nodes (Section 4.1, "LoD Tree Partitioning").
constexpr int kChunkNodes = 2048;
struct Partition {
  int64_t n_sub, n_chunks, n_nodes;
  float4* rec;          // 2 per node, subtree-major: {lo.xyz, node id}, {hi.xyz, meta}
  int32_t* aux;         // per record: first child subtree (bottom internal nodes), else -1
  int32_t* sub_of;      // per node: its subtree
  int32_t* sub_rec;     // per subtree: first record [n_sub + 1]
  int32_t* sub_up;      // per subtree: the tree parent of its root (-1 at the top)
  int32_t* chunk_sub;   // per chunk: first subtree [n_chunks + 1]
  int2* chunk_dep;      // per chunk: the range of earlier chunks holding parents of its subtrees
  uint32_t* stamp;      // per subtree: search epoch when reached or visited
  uint32_t* done;       // per chunk: search epoch when streamed
  int32_t* queue[2];    // subtree queues of the temporal rounds [n_sub each]
  uint32_t* ctr;        // device counters
  uint32_t epoch;       // host: last search epoch
  int max_rounds;       // subtree levels + 1
};

struct Cut {
  uint32_t magic;
  const Scene* scene;
  int64_t n;
  int32_t* F[2];        // frontier buffers (double-buffered so prev == out works)
  int cur;              // index of the buffer holding the latest frontier (-1: none yet)
  int32_t* C;           // cut ids
  int32_t* counts;      // device: [0] |F| of buffer 0, [1] |F| of buffer 1, [2] |C|, [3] |C| copy
  uint32_t* fbits;      // frontier bitmap (kept zero between calls)
  uint32_t* cbits;      // cut bitmap
  int64_t n_words;
  int32_t* q[2];        // level queues of the top-down traversal
  uint32_t* ctr;        // device counters: [0..2] rotating queue counts [3] error
  uint64_t* status;     // compaction: bit counts of every partition (F, C as uint32)
  int64_t n_parts;      // compaction partitions
  uint64_t version;     // counts the cuts written into this handle
};

struct RenderCtx {
  uint32_t magic;
  int64_t max_g, max_pairs;
  int32_t max_w, max_h;
  int64_t max_tiles;
  // projected Gaussians (cut order)
  float4* pg0;          // {mean2d.x, mean2d.y, conic.a, conic.b}
  float4* pg1;          // {conic.c, theta, rho threshold (filter), depth}
  float4* pg2;          // {r, g, b, 0}
  uint4* prec;          // binning record {x0 | y0 << 16, x1 | y1 << 16 (inclusive tile rect),
                        //   kept-tile mask (rect of <= 32 tiles, row-major bits; 0 = big), pair count}
  float* prelax;        // per-Gaussian rounding allowance of the tile test
  uint32_t* big;        // cut positions of Gaussians binned by a whole workgroup
  // depth sort
  uint32_t* dkey[2];
  uint32_t* dval[2];
  uint32_t* offsets;    // first pair of each Gaussian (by cut position)
  // pairs
  uint32_t* tkey[2];
  uint32_t* tval[2];
  uint2* ranges;        // per tile [start, end)
  // per-frame counters, histograms, tickets: zeroed by the setup kernel
  uint32_t* ctr;        // see render.hip for the layout
  uint32_t* hist;       // 6 passes x 256 bins
  uint64_t* status;     // look-back status words (sort passes and scans)
  int64_t status_words;
  uint32_t epoch;
  float* T_final;
  int32_t* n_contrib;
  int32_t* n_eval;
  int32_t* last_contrib;  // tile-list position of the last blended Gaussian, -1 if none
  // what the last frame saved for the backward pass (vy_render with save_state)
  bool saved;             // saved state complete: save_state, no split tiles, exact exponential
  const void* saved_scene;
  const void* saved_cut;
  uint64_t saved_version; // version of that cut
  uint64_t saved_params;  // parameter version of that scene
  vy_camera saved_cam;
  float saved_bg[3];
  // blend planning: tiles split by depth bins
  uint32_t* tile_flag;  // 0 = in tile order, 1 = heavy-first tier, h + 2 = split heavy tile h
  uint32_t* tiers;      // 3 lists of heavy-first tiles
  uint32_t* heavy_list;
  uint32_t* heavy_rec;  // per heavy tile: tile, bins, slot base, bin boundaries and keys
  uint4* jobs;          // (heavy tile, first bin, end bin)
  uint32_t* slot_owner; // heavy tile of each per-bin result slot
  void* pstate_raw;
  uint2* redo;          // (heavy tile, bin) units of the composite's second step
  float4* bin_c;        // per (bin slot, pixel): C_b.rgb, T_b
  int32_t* bin_n;       // per (bin slot, pixel): contributors
  bool split;           // the buffers of split tiles exist
};

uint32_t next_epoch(uint32_t& epoch);   // 24-bit epochs, never 0

// Entry points shared between the library's sources.
// vy_cut_create / vy_render_ctx_create with their one-time initialisation
// enqueued on `st` (`sync`: wait for it, as the public functions do).
int cut_create_on(const vy_scene* scene, void* ws, size_t ws_bytes, hipStream_t st, bool sync, vy_cut** out);
// `split`: with the buffers of tiles split by depth bins (split_min_pairs > 0).
int render_ctx_create_on(int64_t max_g, int32_t max_w, int32_t max_h, int64_t max_pairs, bool split, void* ws,
                         size_t bytes, hipStream_t st, bool sync, vy_render_ctx** out);
size_t render_workspace_bytes(int64_t max_g, int32_t max_w, int32_t max_h, int64_t max_pairs, bool split);
const int32_t* cut_ids_dev(const Cut* c);
const int32_t* cut_count_dev(const Cut* c);            // |C|
const int32_t* cut_frontier_count_dev(const Cut* c);   // |F| of the latest frontier
const uint32_t* cut_err_dev(const Cut* c);             // device-side bound hits of the last cut
// Enqueues the kernel that writes a frame's summary record (32 bytes, see
// vy_frame_stats in vy_serve.h): image hash, cut and pair counts, flags.
// The same record for a frame of the last batch rendered with `batch`.
int batch_frame_finish(const vy_cut* cut, const vy_batch_ctx* batch, const float* image, int32_t width,
                       int32_t height, void* stats, hipStream_t st);
int render_frame_finish(const vy_cut* cut, const vy_render_ctx* ctx, const float* image, int32_t width,
                        int32_t height, void* stats, hipStream_t st);

}  // namespace vy

// --------------------------------------------------------- device helpers ----

#define VY_DEV __device__ __forceinline__

namespace vyd {

VY_DEV uint32_t lane() { return __lane_id(); }
VY_DEV uint64_t ballot(bool p) { return __ballot(p); }
VY_DEV uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

// Relaxed device-scope atomics. No acquire/release ordering is needed where
// they are used: a look-back status word packs its flag and value into one
// 64-bit word (read and written whole), and queue counters written by an
// earlier launch are ordered by the kernel boundary.
template <class T>
VY_DEV T ld_relaxed(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
VY_DEV void st_relaxed(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
VY_DEV T fetch_add(T* p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Look-back status word: [63:40] epoch (24 bit) | [39:38] flag | [37:0] value.
constexpr uint64_t kFlagAgg = 1, kFlagInc = 2;
VY_DEV uint64_t pack_status(uint32_t epoch, uint64_t flag, uint64_t v) {
  return (uint64_t(epoch) << 40) | (flag << 38) | (v & ((1ull << 38) - 1));
}

// Maximum number of polls of a look-back predecessor before giving up (the
// kernel then records an error and continues, so it always terminates).
constexpr uint32_t kSpinLimit = 1u << 22;

// Decoupled look-back (single thread): publishes `aggregate` for partition
// `part`, sums predecessors' values back to the nearest inclusive prefix, and
// publishes the inclusive prefix. Returns the exclusive prefix.
VY_DEV uint64_t lookback(uint64_t* status, uint32_t part, uint32_t stride, uint32_t epoch, uint64_t aggregate,
                         uint32_t* err) {
  uint64_t* me = status + (uint64_t)part * stride;
  if (part == 0) {
    st_relaxed(me, pack_status(epoch, kFlagInc, aggregate));
    return 0;
  }
  st_relaxed(me, pack_status(epoch, kFlagAgg, aggregate));
  uint64_t excl = 0;
  int64_t j = (int64_t)part - 1;
  uint32_t spins = 0;
  while (j >= 0) {
    uint64_t w = ld_relaxed(status + (uint64_t)j * stride);
    uint64_t flag = (w >> 38) & 3ull;
    if ((uint32_t)(w >> 40) != epoch || flag == 0) {
      if (++spins > kSpinLimit) {
        fetch_add(err, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    excl += w & ((1ull << 38) - 1);
    if (flag == kFlagInc) break;
    --j;
  }
  st_relaxed(me, pack_status(epoch, kFlagInc, excl + aggregate));
  return excl;
}

// Decoupled look-back by one whole wave (all 64 lanes call it): lane l polls
// predecessor part-1-l, so each step covers 64 predecessors with independent
// loads instead of one. The nearest inclusive prefix among them ends the walk
// (virtual inclusive 0 before partition 0). Returns the exclusive prefix in
// every lane; lane 0 publishes the aggregate first and the inclusive prefix
// last.
VY_DEV uint64_t lookback_wave(uint64_t* status, uint32_t part, uint32_t stride, uint32_t epoch,
                              uint64_t aggregate, uint32_t* err) {
  const uint32_t l = lane();
  uint64_t* me = status + (uint64_t)part * stride;
  if (part == 0) {
    if (l == 0) st_relaxed(me, pack_status(epoch, kFlagInc, aggregate));
    return 0;
  }
  if (l == 0) st_relaxed(me, pack_status(epoch, kFlagAgg, aggregate));
  uint64_t excl = 0;
  int64_t hi = (int64_t)part - 1;
  uint32_t spins = 0;
  for (;;) {
    const int64_t j = hi - (int64_t)l;
    uint64_t val = 0;
    bool valid = true, inc = true;
    if (j >= 0) {
      const uint64_t w = ld_relaxed(status + (uint64_t)j * stride);
      const uint64_t flag = (w >> 38) & 3ull;
      valid = (uint32_t)(w >> 40) == epoch && flag != 0;
      inc = valid && flag == kFlagInc;
      val = w & ((1ull << 38) - 1);
    }
    const uint64_t inc_m = ballot(inc), bad_m = ballot(!valid);
    const int k = inc_m ? __builtin_ctzll(inc_m) : 64;          // nearest inclusive
    const uint64_t need = k >= 63 ? ~0ull : ((2ull << k) - 1ull);  // lanes 0..k
    if (bad_m & need) {
      if (++spins > kSpinLimit) {
        if (l == 0) fetch_add(err, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    uint64_t v = (int)l <= k ? val : 0ull;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const uint32_t lo = __shfl_xor((uint32_t)v, o, 64), hi32 = __shfl_xor((uint32_t)(v >> 32), o, 64);
      v += ((uint64_t)hi32 << 32) | lo;
    }
    excl += v;
    if (k < 64) break;
    hi -= 64;
  }
  if (l == 0) st_relaxed(me, pack_status(epoch, kFlagInc, excl + aggregate));
  return excl;
}

// First half of a decoupled look-back split in two: publishes partition
// `part`'s aggregate (the inclusive prefix for partition 0).
VY_DEV void publish_aggregate(uint64_t* status, uint32_t part, uint32_t stride, uint32_t epoch, uint64_t aggregate) {
  st_relaxed(status + (uint64_t)part * stride, pack_status(epoch, part == 0 ? kFlagInc : kFlagAgg, aggregate));
}

// Second half, by one thread that polls K predecessors per step with
// independent loads (for the per-digit chains of the radix sort, where every
// thread walks its own chain): sums predecessors' values back to the nearest
// inclusive prefix, publishes the inclusive prefix and returns the exclusive
// one. The aggregate must have been published with publish_aggregate.
template <int K>
VY_DEV uint64_t lookback_poll(uint64_t* status, uint32_t part, uint32_t stride, uint32_t epoch, uint64_t aggregate,
                              uint32_t* err) {
  uint64_t* me = status + (uint64_t)part * stride;
  if (part == 0) return 0;
  uint64_t excl = 0;
  int64_t j = (int64_t)part - 1;
  uint32_t spins = 0;
  while (j >= 0) {
    uint64_t w[K];
#pragma unroll
    for (int i = 0; i < K; ++i) w[i] = j - i >= 0 ? ld_relaxed(status + (uint64_t)(j - i) * stride) : 0ull;
    bool done = false, stall = false;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      if (done || stall || j < 0) continue;
      const uint64_t flag = (w[i] >> 38) & 3ull;
      if ((uint32_t)(w[i] >> 40) != epoch || flag == 0) {
        stall = true;   // poll again from predecessor j
        continue;
      }
      excl += w[i] & ((1ull << 38) - 1);
      if (flag == kFlagInc) done = true;
      else --j;
    }
    if (done) break;
    if (stall) {
      if (++spins > kSpinLimit) {
        fetch_add(err, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  st_relaxed(me, pack_status(epoch, kFlagInc, excl + aggregate));
  return excl;
}

// Block-wide exclusive scan of one uint32 per thread (blockDim == 256).
// `sh` needs 4 (waves) + 1 words. Returns the exclusive prefix; *total = sum.
VY_DEV uint32_t block_excl_scan256(uint32_t v, uint32_t* sh, uint32_t* total) {
  const uint32_t l = lane(), w = threadIdx.x >> 6;
  // wave inclusive scan via DPP-free shuffles
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (l >= (uint32_t)o) x += y;
  }
  if (l == 63) sh[w] = x;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    uint32_t s = sh[i];
    if (i < (int)w) wbase += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return wbase + x - v;
}

}  // namespace vyd
