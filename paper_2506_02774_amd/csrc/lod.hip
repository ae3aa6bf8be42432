// LoD cut kernels (gfx950).
//
// Section 3.1 "Cut Finding": a node is selected when its projected size is
// below tau while its parent's is above. Section 4.1: a full search that visits
// only expanded nodes and their children ("fully-streaming traversal", with
// work dispatched dynamically to whichever wave is free) and the
// temporal-aware search of Algorithm 1, which starts from the previous frame's
// cut and moves each node up (TOP signal) or down (BOTTOM signal) only as far
// as the new camera requires.
//
// Predicate (one device function, compiled without FP contraction so every
// kernel computes the same bits for a node):
//   vis(n)    : the AABB is not entirely outside any of the 4 side planes
//               through the camera centre or the near plane (positive-vertex
//               test on n.(v - pos) >= d);
//   expand(n) : n has children && vis(n) && (fx*ext)^2 > tau^2 * dist^2,
//               ext = longest AABB side, dist = camera centre to AABB.
// Every step of vis and expand is a monotone float32 operation of the AABB
// bounds, so AABB(child) inside AABB(parent) gives expand(child) =>
// expand(parent) exactly; the frontier is then well defined and the temporal
// search reproduces the full search bit for bit.
//
// State kept per cut: the frontier F (non-expanded nodes whose ancestors all
// expand, frustum-culled ones included) and C = F with vis. New F/C are
// collected as bitmaps and compacted to ascending ids (canonical order).
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "vy_common.hpp"

#pragma clang fp contract(off)

namespace {

using namespace vyd;
using vy::kChunkNodes;
using vy::Partition;

struct LodCam {
  float4 pl[5];  // world normal (x, y, z) and offset w: inside iff n.(v - pos) >= w
  float px, py, pz, fx, tau2;
};

VY_DEV bool lod_vis(const float4 a, const float4 b, const LodCam& c) {
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const float4 n = c.pl[k];
    const float vx = n.x >= 0.f ? b.x : a.x;
    const float vy = n.y >= 0.f ? b.y : a.y;
    const float vz = n.z >= 0.f ? b.z : a.z;
    const float s = (n.x * (vx - c.px) + n.y * (vy - c.py)) + n.z * (vz - c.pz);
    if (!(s >= n.w)) return false;
  }
  return true;
}

// a = {lo.xyz, first_child bits}, b = {hi.xyz, parent bits}
VY_DEV bool lod_expand(const float4 a, const float4 b, const LodCam& c, bool& vis) {
  vis = lod_vis(a, b, c);
  const float ext = fmaxf(fmaxf(b.x - a.x, b.y - a.y), b.z - a.z);
  const float dx = fmaxf(fmaxf(a.x - c.px, c.px - b.x), 0.f);
  const float dy = fmaxf(fmaxf(a.y - c.py, c.py - b.y), 0.f);
  const float dz = fmaxf(fmaxf(a.z - c.pz, c.pz - b.z), 0.f);
  const float d2 = (dx * dx + dy * dy) + dz * dz;
  const float fe = c.fx * ext;
  return __float_as_int(a.w) >= 0 && vis && (fe * fe > c.tau2 * d2);
}

VY_DEV void emit_node(int32_t n, bool vis, uint32_t* fbits, uint32_t* cbits) {
  const uint32_t bit = 1u << (n & 31);
  atomicOr(fbits + (n >> 5), bit);
  if (vis) atomicOr(cbits + (n >> 5), bit);
}

// Wave-cooperative emission for (mostly ascending) node ids: runs of lanes
// that hit the same bitmap word are OR-reduced with a segmented shuffle scan
// and written by one atomic per run. Every lane of the wave must call it;
// lanes with active == false contribute nothing.
VY_DEV void emit_wave(bool active, int32_t n, bool vis, uint32_t* fbits, uint32_t* cbits) {
  const int32_t word = active ? (n >> 5) : -1;
  uint32_t fv = active ? (1u << (n & 31)) : 0u;
  uint32_t cv = (active && vis) ? fv : 0u;
  const uint32_t l = lane();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t ow = __shfl_down(word, off, 64);
    const uint32_t of = __shfl_down(fv, off, 64), oc = __shfl_down(cv, off, 64);
    if (l + off < 64 && ow == word) {
      fv |= of;
      cv |= oc;
    }
  }
  const int32_t prev = __shfl_up(word, 1, 64);
  if (active && (l == 0 || prev != word)) {
    atomicOr(fbits + word, fv);
    if (cv) atomicOr(cbits + word, cv);
  }
}

// ctr layout: [0..2] rotating level-queue counters, [3] error count
constexpr int kQ0 = 0, kErr = 3;

__global__ void lod_setup(uint32_t* ctr, int32_t* q0, int seed_root) {
  if (threadIdx.x == 0) {
    ctr[kQ0] = seed_root ? 1u : 0u;
    ctr[kQ0 + 1] = 0;
    ctr[kQ0 + 2] = 0;
    ctr[kErr] = 0;
    if (seed_root) q0[0] = 0;
  }
}

// Exhaustive baseline: every node tests itself and its parent.
// Each wave owns 64 consecutive nodes = 2 whole bitmap words.
__global__ __launch_bounds__(256) void lod_flat(int64_t n, const float4* __restrict__ lod, LodCam cam,
                                                uint32_t* __restrict__ fbits, uint32_t* __restrict__ cbits) {
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t wv = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); wv * 64 < n; wv += nwaves) {
    const int64_t i = wv * 64 + lane();
    bool inF = false, vis = false;
    if (i < n) {
      const float4 a = lod[2 * i], b = lod[2 * i + 1];
      const bool e = lod_expand(a, b, cam, vis);
      bool pe = true;
      const int32_t par = __float_as_int(b.w);
      if (par >= 0) {
        bool pvis;
        pe = lod_expand(lod[2 * (int64_t)par], lod[2 * (int64_t)par + 1], cam, pvis);
      }
      inF = !e && pe;
    }
    const uint64_t mf = ballot(inF), mc = ballot(inF && vis);
    if (lane() == 0) {
      fbits[2 * wv] = (uint32_t)mf;
      cbits[2 * wv] = (uint32_t)mc;
    } else if (lane() == 32) {
      fbits[2 * wv + 1] = (uint32_t)(mf >> 32);
      cbits[2 * wv + 1] = (uint32_t)(mc >> 32);
    }
  }
}

// Block-aggregated append of `push` consecutive ids starting at fc (per
// thread) to a queue: one atomic per block.
VY_DEV void push_children(uint32_t push, int32_t fc, int32_t* q, uint32_t* qcnt, uint32_t cap, uint32_t* err,
                          uint32_t* s_scan, uint32_t* s_tail) {
  uint32_t total;
  const uint32_t off = block_excl_scan256(push, s_scan, &total);
  if (total == 0) return;
  if (threadIdx.x == 0) s_tail[0] = fetch_add(qcnt, total);
  __syncthreads();
  const uint32_t t0 = s_tail[0];
  for (uint32_t k = 0; k < push; ++k) {
    const uint32_t pos = t0 + off + k;
    if (pos < cap) q[pos] = fc + (int32_t)k;
    else fetch_add(err, 1u);
  }
  __syncthreads();
}

// Temporal step (Algorithm 1) for every node of the previous frontier:
//   expand(n)                          -> BOTTOM: descend (children go to the worklist)
//   n != root && !expand(parent(n))    -> TOP: climb to the highest ancestor a with
//                                         !expand(parent(a)) (or the root), emit a
//   otherwise                          -> n stays on the frontier.
__global__ __launch_bounds__(256) void lod_classify(const int32_t* __restrict__ Fprev, const int32_t* n_prev_ptr,
                                                    const float4* __restrict__ lod,
                                                    const int32_t* __restrict__ ccount, LodCam cam,
                                                    int32_t* q0, uint32_t* ctr, uint32_t cap,
                                                    uint32_t* fbits, uint32_t* cbits) {
  __shared__ uint32_t s_scan[8], s_tail[1];
  const int64_t n_prev = *n_prev_ptr;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // uniform trip count so that every thread reaches the block barriers
  const int64_t trips = (n_prev + stride - 1) / stride;
  for (int64_t t = 0; t < trips; ++t) {
    const int64_t i = t * stride + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    uint32_t push = 0;
    int32_t fc = 0;
    const int32_t nd = i < n_prev ? Fprev[i] : -1;
    const bool ok = nd >= 0 && (uint32_t)nd < cap;
    if (i < n_prev && !ok) fetch_add(ctr + kErr, 1u);
    bool em = false, em_vis = false;
    int32_t em_id = 0;
    if (ok) {
      const float4 a = lod[2 * (int64_t)nd], b = lod[2 * (int64_t)nd + 1];
      bool vis;
      if (lod_expand(a, b, cam, vis)) {
        fc = __float_as_int(a.w);
        push = (uint32_t)ccount[nd];
      } else {
        int32_t p = __float_as_int(b.w);
        int32_t cur = nd;
        bool cur_vis = vis;
        // climb while the parent does not expand (bounded by the tree depth limit)
        for (int depth = 0; p >= 0; ++depth) {
          if (depth >= 256) {
            fetch_add(ctr + kErr, 1u);
            break;
          }
          const float4 pa = lod[2 * (int64_t)p], pb = lod[2 * (int64_t)p + 1];
          bool pvis;
          if (lod_expand(pa, pb, cam, pvis)) break;
          cur = p;
          cur_vis = pvis;
          p = __float_as_int(pb.w);
        }
        em = true;
        em_id = cur;
        em_vis = cur_vis;
      }
    }
    emit_wave(em, em_id, em_vis, fbits, cbits);
    push_children(push, fc, q0, ctr + kQ0, cap, ctr + kErr, s_scan, s_tail);
  }
}

// Level launches of the top-down traversal (Section 4.1 "Fully-Streaming LoD
// Tree Traversal": only expanded nodes and their children are visited). Each
// thread takes one queued node and descends up to LEVELS levels on its own (a
// small DFS stack; deeper per-thread descents serialise dependent node loads),
// emitting frontier nodes to the bitmaps; nodes one level deeper are handed to
// the next launch through an LDS buffer that the block appends to the output
// queue with a single atomic. ceil(tree depth / LEVELS) launches cover any
// descent; the last one flags a node it would have to hand on (possible only
// when a fanout above the stack's capacity defers a node early). Launches with
// an empty input queue return at once. Queue counters rotate over three slots:
// launch j reads cnt[j % 3], appends to cnt[(j + 1) % 3] and clears
// cnt[(j + 2) % 3].
constexpr int kLocalLevels = 4;
constexpr int kStack = 16;
constexpr int kOutPerBlock = 256 * 16;

template <int LEVELS>
__global__ __launch_bounds__(256) void lod_level(const int32_t* __restrict__ in_q, uint32_t* cnt3, int j,
                                                 int32_t* __restrict__ out_q, const float4* __restrict__ lod,
                                                 const int32_t* __restrict__ ccount, LodCam cam, uint32_t cap,
                                                 uint32_t* fbits, uint32_t* cbits, uint32_t* err, int last) {
  __shared__ int32_t s_out[kOutPerBlock];
  __shared__ uint32_t s_n, s_base;
  const uint32_t n_in = ld_relaxed(cnt3 + (j % 3));
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt3[(j + 2) % 3] = 0;
  const uint32_t stride = gridDim.x * blockDim.x;
  const uint32_t trips = (n_in + stride - 1) / stride;
  uint32_t* out_cnt = cnt3 + ((j + 1) % 3);
  for (uint32_t t = 0; t < trips; ++t) {
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    const uint32_t i = t * stride + blockIdx.x * blockDim.x + threadIdx.x;
    int32_t stk[kStack];
    int32_t dep[kStack];
    int sp = 0;
    if (i < n_in) {
      const int32_t nd = in_q[i];
      if (nd >= 0 && (uint32_t)nd < cap) {
        stk[0] = nd;
        dep[0] = 0;
        sp = 1;
      } else {
        fetch_add(err, 1u);
      }
    }
    while (sp > 0) {
      --sp;
      const int32_t n = stk[sp], d = dep[sp];
      const float4 a = lod[2 * (int64_t)n], b = lod[2 * (int64_t)n + 1];
      bool vis;
      if (!lod_expand(a, b, cam, vis)) {
        emit_node(n, vis, fbits, cbits);
        continue;
      }
      const int32_t fc = __float_as_int(a.w), cc = ccount[n];
      for (int k = cc - 1; k >= 0; --k) {
        const int32_t ch = fc + k;
        if (d + 1 < LEVELS && sp < kStack) {
          stk[sp] = ch;
          dep[sp] = d + 1;
          ++sp;
        } else if (last) {
          fetch_add(err, 1u);   // deeper than the launches cover: the cut would be incomplete
        } else {
          const uint32_t slot = atomicAdd(&s_n, 1u);
          if (slot < (uint32_t)kOutPerBlock) {
            s_out[slot] = ch;
          } else {
            const uint32_t g = fetch_add(out_cnt, 1u);
            if (g < cap) out_q[g] = ch;
            else fetch_add(err, 1u);
          }
        }
      }
    }
    __syncthreads();
    const uint32_t nl = s_n < (uint32_t)kOutPerBlock ? s_n : (uint32_t)kOutPerBlock;
    if (threadIdx.x == 0) s_base = nl ? fetch_add(out_cnt, nl) : 0u;
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < nl; k += blockDim.x) {
      const uint32_t pos = s_base + k;
      if (pos < cap) out_q[pos] = s_out[k];
      else fetch_add(err, 1u);
    }
    __syncthreads();
  }
}

// Level launches with a workgroup-local breadth-first walk (Section 4.1,
// "Fully-Streaming LoD Tree Traversal"). A workgroup takes SEEDS queued nodes
// at a time and walks their subtrees level by level for LEVELS levels, with
// each level's frontier in LDS and one node per thread: a level costs one
// dependent record load per thread instead of one per node of a per-thread
// descent. SEEDS << (LEVELS - 1) frontier slots hold every node of a binary
// tree's LEVELS levels (wider fanouts that overflow them queue the extra
// nodes for the next launch). The children of the last level are queued for
// the next launch with one atomic per 256 nodes. ceil(tree depth / LEVELS)
// launches cover any descent, and the last one flags a node it would have to
// queue. Queue counters rotate over three slots as in lod_level.
constexpr int kBfsLevels = 13, kBfsSeeds = 1, kBfsSlots = kBfsSeeds << (kBfsLevels - 1);

__global__ __launch_bounds__(256) void lod_bfs(const int32_t* __restrict__ in_q, uint32_t* cnt3, int j,
                                               int32_t* __restrict__ out_q, const float4* __restrict__ lod,
                                               const int32_t* __restrict__ ccount, LodCam cam, uint32_t cap,
                                               uint32_t* fbits, uint32_t* cbits, uint32_t* err, int last) {
  __shared__ int32_t s_f[2][kBfsSlots];
  __shared__ uint32_t s_n[2], s_scan[8], s_tail[1];
  const uint32_t n_in = ld_relaxed(cnt3 + (j % 3));
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt3[(j + 2) % 3] = 0;
  uint32_t* out_cnt = cnt3 + ((j + 1) % 3);
  const uint32_t tid = threadIdx.x;
  const uint32_t nchunks = (n_in + kBfsSeeds - 1) / kBfsSeeds;
  for (uint32_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const uint32_t c0 = chunk * kBfsSeeds;
    const uint32_t ns = n_in - c0 < (uint32_t)kBfsSeeds ? n_in - c0 : (uint32_t)kBfsSeeds;
    if (tid < ns) {
      int32_t nd = in_q[c0 + tid];
      if (nd < 0 || (uint32_t)nd >= cap) {
        fetch_add(err, 1u);
        nd = -1;
      }
      s_f[0][tid] = nd;
    }
    if (tid == 0) {
      s_n[0] = ns;
      s_n[1] = 0;
    }
    __syncthreads();
    int cur = 0;
    for (int d = 0; d < kBfsLevels; ++d) {
      const uint32_t nc = s_n[cur] < (uint32_t)kBfsSlots ? s_n[cur] : (uint32_t)kBfsSlots;
      if (nc == 0) break;   // uniform: read after the barrier
      const bool deepest = d + 1 == kBfsLevels;
      // rounds of 256 nodes (a uniform trip count: the last level's queueing uses block barriers)
      for (uint32_t r0 = 0; r0 < nc; r0 += blockDim.x) {
        const uint32_t t = r0 + tid;
        const int32_t n = t < nc ? s_f[cur][t] : -1;
        uint32_t push = 0;
        int32_t fc = 0;
        if (n >= 0) {
          const float4 a = lod[2 * (int64_t)n], b = lod[2 * (int64_t)n + 1];
          bool vis;
          if (!lod_expand(a, b, cam, vis)) {
            emit_node(n, vis, fbits, cbits);
          } else {
            fc = __float_as_int(a.w);
            const int32_t cc = ccount[n];
            if (deepest) {
              push = (uint32_t)cc;
            } else {
              for (int k = 0; k < cc; ++k) {
                const uint32_t slot = atomicAdd(&s_n[cur ^ 1], 1u);
                if (slot < (uint32_t)kBfsSlots) {
                  s_f[cur ^ 1][slot] = fc + k;
                } else if (last) {
                  fetch_add(err, 1u);
                } else {
                  const uint32_t g = fetch_add(out_cnt, 1u);   // past the slots (fanout above 2): next launch
                  if (g < cap) out_q[g] = fc + k;
                  else fetch_add(err, 1u);
                }
              }
            }
          }
        }
        if (deepest) {
          if (last) {
            if (push) fetch_add(err, 1u);   // deeper than the launches cover: the cut would be incomplete
          } else {
            push_children(push, fc, out_q, out_cnt, cap, err, s_scan, s_tail);
          }
        }
      }
      __syncthreads();
      if (tid == 0) s_n[cur] = 0;
      cur ^= 1;
      __syncthreads();
    }
    // a level loop that ended on an empty level (nc == 0) ran no barrier after
    // its read of s_n: the next chunk's seeding must not overwrite s_n or s_f
    // before every wave has read them
    __syncthreads();
  }
}

// Compaction of the F and C bitmaps into ascending ids over partitions of
// 768 words, zeroing the bitmaps as they are read: a first launch counts
// every partition's bits, and each partition of the second sums the counts
// of the partitions before it (at most a few thousand words, read from L2)
// instead of waiting on a look-back chain across the partitions.
// A partition is read as 3 rounds of 256 consecutive words (one per thread);
// each wave gathers its words' ids of a round in LDS, as 16-bit offsets into
// the partition, and writes them out with coalesced stores.
// The 6 per-thread counts (2 bitmaps x 3 rounds, each <= 32) are scanned in
// one pass as 16-bit fields of 4 words (a round's totals stay below 2^16).
// 3 words per thread: 1465 partitions of 24576 nodes for a 36M-node tree,
// all resident at once, with the densest partition's ids spread over
// fewer words than with 4 (1099 partitions) or 2 (2198, a second round)
constexpr int kWordsPerThread = 3, kWordsPerPart = 256 * kWordsPerThread;
static_assert(kWordsPerThread <= 4, "lod_compact packs two words' counts per 16-bit pair of a uint4 field");
static_assert(kWordsPerPart * 32 <= 65536, "lod_compact stages a partition's ids as 16-bit offsets");

VY_DEV uint4 block_excl_scan256_x4(uint4 v, uint4* sh, uint4* total) {
  const uint32_t l = lane(), w = threadIdx.x >> 6;
  uint4 x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint4 y = make_uint4(__shfl_up(x.x, o, 64), __shfl_up(x.y, o, 64), __shfl_up(x.z, o, 64),
                               __shfl_up(x.w, o, 64));
    if (l >= (uint32_t)o) {
      x.x += y.x;
      x.y += y.y;
      x.z += y.z;
      x.w += y.w;
    }
  }
  if (l == 63) sh[w] = x;
  __syncthreads();
  uint4 wb = make_uint4(0, 0, 0, 0), tot = make_uint4(0, 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint4 t = sh[i];
    if (i < (int)w) {
      wb.x += t.x;
      wb.y += t.y;
      wb.z += t.z;
      wb.w += t.w;
    }
    tot.x += t.x;
    tot.y += t.y;
    tot.z += t.z;
    tot.w += t.w;
  }
  __syncthreads();
  *total = tot;
  return make_uint4(wb.x + x.x - v.x, wb.y + x.y - v.y, wb.z + x.z - v.z, wb.w + x.w - v.w);
}

// Frontier and cut bit counts of every compaction partition, so that a
// partition's output offset is a plain sum over the partitions before it.
__global__ __launch_bounds__(256) void lod_part_totals(int64_t n_words, const uint32_t* __restrict__ fbits,
                                                       const uint32_t* __restrict__ cbits,
                                                       uint32_t* __restrict__ part_tot) {
  __shared__ uint32_t s_sum[2];
  if (threadIdx.x < 2) s_sum[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kWordsPerPart;
  uint32_t a = 0u, b = 0u;
#pragma unroll
  for (int k = 0; k < kWordsPerThread; ++k) {
    const int64_t w = base + k * 256 + threadIdx.x;
    if (w < n_words) {
      a += (uint32_t)__popc(fbits[w]);
      b += (uint32_t)__popc(cbits[w]);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  if (lane() == 0) {
    atomicAdd(&s_sum[0], a);
    atomicAdd(&s_sum[1], b);
  }
  __syncthreads();
  if (threadIdx.x < 2) part_tot[2 * (int64_t)blockIdx.x + threadIdx.x] = s_sum[threadIdx.x];
}

__global__ __launch_bounds__(256) void lod_compact(int64_t n_words, uint32_t* __restrict__ fbits,
                                                   uint32_t* __restrict__ cbits, int32_t* __restrict__ Fout,
                                                   int32_t* __restrict__ Cout, int32_t* counts, int f_slot,
                                                   const uint32_t* __restrict__ part_tot, uint32_t n_parts) {
  __shared__ uint4 s_scan4[4];
  __shared__ uint32_t s_ex[2];
  // ids staged as 16-bit offsets into the partition's 32768 node ids: 16 KB,
  // so that every partition of a large tree is resident at once
  __shared__ uint16_t s_ids[256 * 32];
  const uint32_t part = blockIdx.x;
  if (threadIdx.x < 2) s_ex[threadIdx.x] = 0u;
  // the partition's bitmap words, in flight while the offsets are summed
  const int64_t base = (int64_t)part * kWordsPerPart;
  uint32_t wd[2][kWordsPerThread];
#pragma unroll
  for (int k = 0; k < kWordsPerThread; ++k) {
    const int64_t w = base + k * 256 + threadIdx.x;
    wd[0][k] = w < n_words ? fbits[w] : 0u;
    wd[1][k] = w < n_words ? cbits[w] : 0u;
  }
  __syncthreads();
  {
    // the offsets of this partition's ids: totals of the partitions before it,
    // eight loads per thread in flight at a time
    const uint2* __restrict__ pt = reinterpret_cast<const uint2*>(part_tot);
    uint32_t pa = 0u, pb = 0u;
    for (uint32_t j0 = threadIdx.x; j0 < part; j0 += 256 * 8) {
      uint2 t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint32_t j = j0 + 256u * u;
        t[u] = j < part ? pt[j] : make_uint2(0u, 0u);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        pa += t[u].x;
        pb += t[u].y;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      pa += __shfl_xor(pa, o, 64);
      pb += __shfl_xor(pb, o, 64);
    }
    if (lane() == 0) {
      atomicAdd(&s_ex[0], pa);
      atomicAdd(&s_ex[1], pb);
    }
  }
  // fields: .x = F rounds 0 | 1 << 16, .y = F round 2 (| 3 << 16 with 4 rounds), .z/.w the same for C
  uint32_t f4[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int k = 0; k < kWordsPerThread; ++k) f4[2 * q + (k >> 1)] |= (uint32_t)__popc(wd[q][k]) << (16 * (k & 1));
  const uint4 cnt4 = make_uint4(f4[0], f4[1], f4[2], f4[3]);
  uint4 tot4;
  const uint4 off4 = block_excl_scan256_x4(cnt4, s_scan4, &tot4);
  uint32_t off[2][kWordsPerThread], rt[2][kWordsPerThread], tot[2];
  {
    const uint32_t o[4] = {off4.x, off4.y, off4.z, off4.w}, t[4] = {tot4.x, tot4.y, tot4.z, tot4.w};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
#pragma unroll
      for (int k = 0; k < kWordsPerThread; ++k) {
        off[q][k] = (o[2 * q + (k >> 1)] >> (16 * (k & 1))) & 0xFFFFu;
        rt[q][k] = (t[2 * q + (k >> 1)] >> (16 * (k & 1))) & 0xFFFFu;
      }
      tot[q] = 0u;
#pragma unroll
      for (int k = 0; k < kWordsPerThread; ++k) tot[q] += rt[q][k];
    }
  }
  __syncthreads();
  // each wave stages the ids of its 64 words of a round in its own LDS slice
  // and writes them as one contiguous, coalesced range: no workgroup barriers
  const uint32_t ln = lane();
  uint16_t* slice = s_ids + (threadIdx.x >> 6) * (64 * 32);
  const int32_t id0 = (int32_t)(base * 32);   // the partition's first node id
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    int32_t* out = (q == 0 ? Fout : Cout) + s_ex[q];
    uint32_t r0 = 0;   // ids of the partition before this round
#pragma unroll
    for (int k = 0; k < kWordsPerThread; ++k) {
      const int64_t w = base + k * 256 + threadIdx.x;
      uint32_t m = wd[q][k];
      // the wave's first offset (lane 0's: the scan is ascending over threads)
      // and its id count (the last lane's offset plus its bits)
      const uint32_t o0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)off[q][k]);
      const uint32_t oe = off[q][k] + (uint32_t)__popc(m);
      const uint32_t n = (uint32_t)__builtin_amdgcn_readlane((int)oe, 63) - o0;
      uint32_t o = off[q][k] - o0;
      const uint32_t wl = (uint32_t)(k * 256 + threadIdx.x) * 32u;   // the word's first local id
      if (m == 0xFFFFFFFFu) {
        // a full word (dense parts of the cut): its 32 consecutive ids at once
#pragma unroll
        for (int b = 0; b < 32; ++b) slice[o + b] = (uint16_t)(wl + (uint32_t)b);
      } else {
        while (m) {
          const int b = __ffs(m) - 1;
          m &= m - 1;
          slice[o++] = (uint16_t)(wl + (uint32_t)b);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // the staged range to memory, four LDS reads per lane in flight
      int32_t* dst = out + r0 + o0;
      uint32_t i = ln;
      for (; i + 192u < n; i += 256u) {
        const int32_t a0 = slice[i], a1 = slice[i + 64u], a2 = slice[i + 128u], a3 = slice[i + 192u];
        dst[i] = id0 + a0;
        dst[i + 64u] = id0 + a1;
        dst[i + 128u] = id0 + a2;
        dst[i + 192u] = id0 + a3;
      }
      for (; i < n; i += 64u) dst[i] = id0 + (int32_t)slice[i];
      r0 += rt[q][k];
      if (wd[q][k]) (q == 0 ? fbits : cbits)[w] = 0u;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  if (part == n_parts - 1 && threadIdx.x == 0) {
    counts[f_slot] = (int32_t)(s_ex[0] + tot[0]);
    counts[2] = (int32_t)(s_ex[1] + tot[1]);
  }
}

// ------------------------------------------------ subtree-chunk traversal ----
//
// Section 4.1 on a partition of the tree (Partition, built once per scene by
// vy_scene_partition): height-2 subtrees in BFS order, stored subtree after
// subtree, packed into chunks of consecutive subtrees of at most kChunkNodes
// nodes. Record meta bits: [0, 8) local index of the parent within the
// subtree (255 at the subtree's root), 8 internal node, 9 bottom node (its
// children root other subtrees), [10, 21) the subtree's index within its
// chunk, [21, 32) the number of children (up to 2047).
//
// Full search ("Fully-Streaming LoD Tree Traversal"): persistent workgroups
// take chunks in BFS order from an atomic ticket. A chunk waits until the
// chunks holding the parents of its subtrees are done, streams its records
// into LDS with coalesced loads, and evaluates the subtrees that are reached
// (the root's subtree, or one whose root's parent expands: stamped with the
// search's epoch by the parent's chunk). Within a subtree a node is on the
// frontier when it does not expand and its parent in the subtree does (or it
// is the subtree's root); an expanding bottom node stamps its children's
// subtrees as reached. The search ends as soon as every reached subtree has
// been evaluated: a clean cut then separates the top of the tree from the
// bottom, and the remaining chunks are skipped.
//
// Temporal search (Algorithm 1 per subtree): the subtrees holding the nodes of
// the previous frontier are evaluated; a subtree whose root's parent does not
// expand signals TOP (its local result is dropped and its parent subtree is
// queued, once), an expanding bottom node signals BOTTOM (its children's
// subtrees are queued, once); the others give their local frontier nodes.
// Rounds of one launch each run until the queue is empty.
constexpr uint32_t kMetaRootParent = 255u;
constexpr int kChunkCtrTicket = 0, kChunkCtrReached = 1, kChunkCtrFinished = 2,
              kChunkCtrQ = 4;   // 4..6: rotating round-queue counts
constexpr int kMaxSubNodes = 64;   // a subtree's nodes fit a 64-bit mask (fanout <= 7)

VY_DEV bool rec_expand(float4 a, float4 b, const LodCam& cam, bool& vis) {
  const uint32_t meta = __float_as_uint(b.w);
  const float4 a2 = make_float4(a.x, a.y, a.z, __int_as_float(((meta >> 8) & 1u) ? 0 : -1));
  return lod_expand(a2, b, cam, vis);
}

__global__ void lod_chunk_setup(uint32_t* ctr, uint32_t* stamp, uint32_t epoch, int full) {
  if (threadIdx.x == 0) {
    ctr[kChunkCtrTicket] = 0;
    ctr[kChunkCtrReached] = full ? 1u : 0u;
    ctr[kChunkCtrFinished] = 0;
    ctr[kChunkCtrQ] = ctr[kChunkCtrQ + 1] = ctr[kChunkCtrQ + 2] = 0;
    if (full) stamp[0] = epoch;   // the root's subtree is reached
  }
}

struct ChunkArgs {
  const float4* rec;
  const int32_t* aux;
  const int32_t* sub_rec;
  const int32_t* sub_up;
  const int32_t* sub_of;
  const int32_t* chunk_sub;
  const int2* chunk_dep;
  uint32_t* stamp;
  uint32_t* done;
  uint32_t* ctr;
  int32_t* queue0;
  int32_t* queue1;
  int64_t n_chunks, n_sub;
};

__global__ __launch_bounds__(256) void lod_chunk_stream(ChunkArgs P, LodCam cam, uint32_t epoch,
                                                        uint32_t* __restrict__ fbits, uint32_t* __restrict__ cbits,
                                                        uint32_t* err) {
  __shared__ float4 s_a[kChunkNodes], s_b[kChunkNodes];
  __shared__ uint16_t s_first[kChunkNodes + 1];   // first record of each subtree of the chunk
  __shared__ uint8_t s_flag[kChunkNodes];         // 1 evaluated, 2 expands, 4 visible, 8 emitted
  __shared__ uint8_t s_reached[kChunkNodes];      // per subtree of the chunk
  __shared__ uint32_t s_c, s_go, s_changed, s_any, s_eval, s_reach;
  const uint32_t tid = threadIdx.x;
  for (;;) {
    if (tid == 0) {
      s_c = fetch_add(P.ctr + kChunkCtrTicket, 1u);
      // every reached subtree evaluated already: nothing further down is reachable
      const uint32_t fin = ld_relaxed(P.ctr + kChunkCtrFinished);
      __threadfence();
      const uint32_t rea = ld_relaxed(P.ctr + kChunkCtrReached);
      s_go = fin != rea ? 1u : 0u;
    }
    __syncthreads();
    const uint32_t c = s_c;
    if (c >= (uint32_t)P.n_chunks) break;
    if (!s_go) {
      if (tid == 0) st_relaxed(P.done + c, epoch);
      break;
    }
    // wait for the chunks that hold the parents of this chunk's subtrees
    if (tid == 0) {
      const int2 dep = P.chunk_dep[c];
      for (int d = dep.x; d <= dep.y; ++d) {
        uint32_t spins = 0;
        while (ld_relaxed(P.done + d) != epoch) {
          if (++spins > (1u << 20)) {
            fetch_add(err, 1u);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      __threadfence();
      s_any = 0;
      s_eval = 0;
      s_reach = 0;
    }
    __syncthreads();
    const int32_t s0 = P.chunk_sub[c], s1 = P.chunk_sub[c + 1];
    const int32_t r0 = P.sub_rec[s0], nrec = P.sub_rec[s1] - r0;
    for (int j = tid; j <= s1 - s0; j += blockDim.x) {
      s_first[j] = (uint16_t)(P.sub_rec[s0 + j] - r0);
      if (j < s1 - s0) {
        const bool rch = ld_relaxed(P.stamp + s0 + j) == epoch;
        s_reached[j] = rch ? 1 : 0;
        if (rch) s_any = 1;
      }
    }
    __syncthreads();
    if (s_any) {
      for (int k = tid; k < nrec; k += blockDim.x) {   // stream the chunk's records into LDS
        s_a[k] = P.rec[2 * (int64_t)(r0 + k)];
        s_b[k] = P.rec[2 * (int64_t)(r0 + k) + 1];
        s_flag[k] = 0;
      }
      uint32_t my_eval = 0, my_reach = 0;
      const int trips = (nrec + (int)blockDim.x - 1) / (int)blockDim.x;
      // passes: a subtree reached from a parent in this chunk is evaluated in the next pass
      for (;;) {
        __syncthreads();
        if (tid == 0) s_changed = 0;
        for (int k = tid; k < nrec; k += blockDim.x) {
          const uint32_t meta = __float_as_uint(s_b[k].w);
          if (s_reached[(meta >> 10) & 2047u] && !(s_flag[k] & 1u)) {
            bool vis;
            const bool e = rec_expand(s_a[k], s_b[k], cam, vis);
            s_flag[k] = (uint8_t)(1u | (e ? 2u : 0u) | (vis ? 4u : 0u));
          }
        }
        __syncthreads();
        for (int t = 0; t < trips; ++t) {
          const int k = t * (int)blockDim.x + (int)tid;
          bool em = false, em_vis = false;
          int32_t id = 0;
          if (k < nrec && (s_flag[k] & 9u) == 1u) {
            s_flag[k] |= 8u;
            const uint32_t meta = __float_as_uint(s_b[k].w);
            const uint32_t lp = meta & 255u, j = (meta >> 10) & 2047u;
            const bool e = (s_flag[k] & 2u) != 0;
            if (lp == kMetaRootParent) ++my_eval;
            const bool pe = lp == kMetaRootParent || (s_flag[s_first[j] + lp] & 2u);
            if (!e && pe) {
              em = true;
              id = __float_as_int(s_a[k].w);
              em_vis = (s_flag[k] & 4u) != 0;
            }
            if (e && ((meta >> 9) & 1u)) {   // BOTTOM: the children's subtrees are reached
              const uint32_t cnt = meta >> 21;
              const int32_t cs0 = P.aux[r0 + k];
              for (uint32_t i = 0; i < cnt; ++i) {
                const int32_t cs = cs0 + (int32_t)i;
                if (cs < s1) {
                  s_reached[cs - s0] = 1;
                  s_changed = 1;
                } else {
                  st_relaxed(P.stamp + cs, epoch);
                }
              }
              my_reach += cnt;
            }
          }
          emit_wave(em, id, em_vis, fbits, cbits);
        }
        __syncthreads();
        if (!s_changed) break;
      }
      if (my_eval) atomicAdd(&s_eval, my_eval);
      if (my_reach) atomicAdd(&s_reach, my_reach);
      __syncthreads();
      if (tid == 0) {
        // reached before finished: a reader that sees finished == reached sees no work left
        __threadfence();
        if (s_reach) fetch_add(P.ctr + kChunkCtrReached, s_reach);
        __threadfence();
        if (s_eval) fetch_add(P.ctr + kChunkCtrFinished, s_eval);
      }
    }
    if (tid == 0) {
      __threadfence();
      st_relaxed(P.done + c, epoch);
    }
    __syncthreads();
  }
}

// Wave-aggregated append of one id per pushing lane.
VY_DEV void push_wave(bool push, int32_t id, int32_t* q, uint32_t* qcnt, uint32_t cap, uint32_t* err) {
  const uint64_t m = ballot(push);
  if (!m) return;
  const uint32_t leader = (uint32_t)__builtin_ctzll(m);
  uint32_t base = 0;
  if (lane() == leader) base = fetch_add(qcnt, (uint32_t)__popcll(m));
  base = __shfl(base, (int)leader, 64);
  if (push) {
    const uint32_t pos = base + (uint32_t)__popcll(m & lanemask_lt());
    if (pos < cap) q[pos] = id;
    else fetch_add(err, 1u);
  }
}

// The subtrees of the previous frontier's nodes, each queued once.
__global__ __launch_bounds__(256) void lod_sub_identify(ChunkArgs P, const int32_t* __restrict__ Fprev,
                                                        const int32_t* n_prev_ptr, uint32_t epoch, uint32_t cap_nodes,
                                                        uint32_t* err) {
  const int64_t n_prev = *n_prev_ptr;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t trips = (n_prev + stride - 1) / stride;
  for (int64_t t = 0; t < trips; ++t) {
    const int64_t i = t * stride + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool push = false;
    int32_t sid = 0;
    if (i < n_prev) {
      const int32_t nd = Fprev[i];
      if (nd < 0 || (uint32_t)nd >= cap_nodes) {
        fetch_add(err, 1u);
      } else {
        sid = P.sub_of[nd];
        push = atomicExch(P.stamp + sid, epoch) != epoch;
      }
    }
    push_wave(push, sid, P.queue0, P.ctr + kChunkCtrQ, (uint32_t)P.n_sub, err);
  }
}

// One round of Algorithm 1 over queued subtrees (one thread per subtree).
__global__ __launch_bounds__(256) void lod_sub_round(ChunkArgs P, const float4* __restrict__ lod, LodCam cam,
                                                     uint32_t epoch, int j, int last, uint32_t* __restrict__ fbits,
                                                     uint32_t* __restrict__ cbits, uint32_t* err) {
  uint32_t* cnt3 = P.ctr + kChunkCtrQ;
  const uint32_t n_in = ld_relaxed(cnt3 + (j % 3));
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt3[(j + 2) % 3] = 0;
  uint32_t* out_cnt = cnt3 + ((j + 1) % 3);
  const int32_t* in_q = (j & 1) ? P.queue1 : P.queue0;
  int32_t* out_q = (j & 1) ? P.queue0 : P.queue1;
  const uint32_t stride = gridDim.x * blockDim.x;
  const uint32_t trips = (n_in + stride - 1) / stride;
  for (uint32_t t = 0; t < trips; ++t) {
    const uint32_t i = t * stride + blockIdx.x * blockDim.x + threadIdx.x;
    int32_t top = -1;                 // TOP: the parent subtree to queue
    int32_t bot_first = -1;           // BOTTOM: children's subtrees to queue, in runs
    if (i < n_in) {
      const int32_t sid = in_q[i];
      const int32_t rs = P.sub_rec[sid], m = P.sub_rec[sid + 1] - rs;
      const int32_t up = P.sub_up[sid];
      bool clean = up < 0;
      if (!clean) {
        bool pvis;
        clean = lod_expand(lod[2 * (int64_t)up], lod[2 * (int64_t)up + 1], cam, pvis);
      }
      if (!clean) {
        const int32_t ps = P.sub_of[up];
        if (atomicExch(P.stamp + ps, epoch) != epoch) top = ps;
      } else {
        uint64_t emask = 0;
        for (int k = 0; k < m && k < kMaxSubNodes; ++k) {
          const float4 a = P.rec[2 * (int64_t)(rs + k)], b = P.rec[2 * (int64_t)(rs + k) + 1];
          const uint32_t meta = __float_as_uint(b.w);
          const uint32_t lp = meta & 255u;
          bool vis;
          const bool e = rec_expand(a, b, cam, vis);
          const bool pe = lp == kMetaRootParent || ((emask >> lp) & 1ull);
          if (e) emask |= 1ull << k;
          if (!e && pe) emit_node(__float_as_int(a.w), vis, fbits, cbits);
          if (e && ((meta >> 9) & 1u)) {
            const uint32_t cnt = meta >> 21;
            const int32_t cs0 = P.aux[rs + k];
            for (uint32_t q = 0; q < cnt; ++q) {
              const int32_t cs = cs0 + (int32_t)q;
              if (atomicExch(P.stamp + cs, epoch) != epoch) {
                if (last) {
                  fetch_add(err, 1u);   // deeper than the rounds cover
                } else {
                  const uint32_t pos = fetch_add(out_cnt, 1u);
                  if (pos < (uint32_t)P.n_sub) out_q[pos] = cs;
                  else fetch_add(err, 1u);
                }
              }
            }
          }
        }
        (void)bot_first;
      }
    }
    if (last) {
      if (top >= 0) fetch_add(err, 1u);
    } else {
      push_wave(top >= 0, top, out_q, out_cnt, (uint32_t)P.n_sub, err);
    }
  }
}

__global__ void fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void set_count(int32_t* p, int32_t v) {
  if (threadIdx.x == 0) p[0] = v;
}

LodCam make_cam(const vy_camera* c, float tau) {
  LodCam L;
  const float* R = c->R;
  const float W = (float)c->width, H = (float)c->height;
  const float nc[5][3] = {{c->fx, 0.f, c->cx}, {-c->fx, 0.f, W - c->cx}, {0.f, c->fy, c->cy},
                          {0.f, -c->fy, H - c->cy}, {0.f, 0.f, 1.f}};
  for (int p = 0; p < 5; ++p) {
    float n[3];
    for (int k = 0; k < 3; ++k) n[k] = (nc[p][0] * R[0 + k] + nc[p][1] * R[3 + k]) + nc[p][2] * R[6 + k];
    L.pl[p] = make_float4(n[0], n[1], n[2], p == 4 ? c->znear : 0.f);
  }
  L.px = c->pos[0];
  L.py = c->pos[1];
  L.pz = c->pos[2];
  L.fx = c->fx;
  L.tau2 = tau * tau;
  return L;
}

}  // namespace

using namespace vy;

extern "C" {

size_t vy_cut_workspace_bytes(int64_t n) {
  if (n < 1) return 0;
  const int64_t n_words = (n + 31) / 32 + 64;
  const int64_t n_parts = (n_words + kWordsPerPart - 1) / kWordsPerPart;
  return (size_t)n * 4 * 5        // F[2], C, two level queues
         + (size_t)n_words * 4 * 2 // bitmaps
         + 64 * 4 + 64 * 4         // counts, ctr
         + (size_t)n_parts * 16    // per-partition bit counts
         + 16 * 256;               // alignment slack
}

int vy_cut_create(const vy_scene* scene, void* ws, size_t ws_bytes, vy_cut** out) {
  return vy::cut_create_on(scene, ws, ws_bytes, nullptr, true, out);
}

}  // extern "C"

namespace vy {

// vy_cut_create with the initialisation enqueued on `st`; `sync` waits for it.
int cut_create_on(const vy_scene* scene, void* ws, size_t ws_bytes, hipStream_t st, bool sync, vy_cut** out) {
  const Scene* s = (const Scene*)scene;
  if (!s || s->magic != kSceneMagic || !ws || !out) return fail(VY_ERR_ARG, "vy_cut_create: bad argument");
  if (ws_bytes < vy_cut_workspace_bytes(s->n))
    return fail(VY_ERR_ARG, "vy_cut_create: workspace %zu < %zu bytes", ws_bytes, vy_cut_workspace_bytes(s->n));
  Cut* c = (Cut*)calloc(1, sizeof(Cut));
  if (!c) return fail(VY_ERR_ARG, "vy_cut_create: out of host memory");
  Carver cv(ws, ws_bytes);
  c->magic = kCutMagic;
  c->scene = s;
  c->n = s->n;
  c->n_words = (s->n + 31) / 32 + 64;
  c->n_parts = (c->n_words + kWordsPerPart - 1) / kWordsPerPart;
  c->F[0] = cv.take<int32_t>(s->n);
  c->F[1] = cv.take<int32_t>(s->n);
  c->C = cv.take<int32_t>(s->n);
  c->q[0] = cv.take<int32_t>(s->n);
  c->q[1] = cv.take<int32_t>(s->n);
  c->fbits = cv.take<uint32_t>(c->n_words);
  c->cbits = cv.take<uint32_t>(c->n_words);
  c->counts = cv.take<int32_t>(64);
  c->ctr = cv.take<uint32_t>(64);
  c->status = cv.take<uint64_t>(2 * c->n_parts);
  c->cur = -1;
  if (!cv.ok()) {
    free(c);
    return fail(VY_ERR_ARG, "vy_cut_create: workspace layout overflow");
  }
  // one-time initialisation: bitmaps, counters and partition counts zero
  hipError_t e = hipMemsetAsync(c->fbits, 0, sizeof(uint32_t) * c->n_words, st);
  if (e == hipSuccess) e = hipMemsetAsync(c->cbits, 0, sizeof(uint32_t) * c->n_words, st);
  if (e == hipSuccess) e = hipMemsetAsync(c->counts, 0, 64 * 4, st);
  if (e == hipSuccess) e = hipMemsetAsync(c->ctr, 0, 64 * 4, st);
  if (e == hipSuccess) e = hipMemsetAsync(c->status, 0, 16 * c->n_parts, st);
  if (e == hipSuccess && sync) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free(c);
    return fail(VY_ERR_HIP, "vy_cut_create: %s", hipGetErrorString(e));
  }
  *out = (vy_cut*)c;
  return VY_OK;
}

}  // namespace vy

extern "C" {

int vy_cut_free(vy_cut* cut) {
  Cut* c = (Cut*)cut;
  if (!c) return VY_OK;
  if (c->magic != kCutMagic) return fail(VY_ERR_ARG, "vy_cut_free: not a cut");
  c->magic = 0;
  free(c);
  return VY_OK;
}

int vy_lod_cut(const vy_scene* scene, const vy_camera* cam, float tau, vy_cut* prev, vy_cut* out, int full_mode,
               void* stream) {
  const Scene* s = (const Scene*)scene;
  Cut* o = (Cut*)out;
  Cut* p = (Cut*)prev;
  if (!s || s->magic != kSceneMagic || !cam || !o || o->magic != kCutMagic)
    return fail(VY_ERR_ARG, "vy_lod_cut: bad argument");
  if (o->scene != s) return fail(VY_ERR_ARG, "vy_lod_cut: output cut belongs to another scene");
  if (!(tau >= 0.f) || cam->width < 1 || cam->height < 1 || !(cam->fx > 0.f) || !(cam->fy > 0.f))
    return fail(VY_ERR_ARG, "vy_lod_cut: invalid tau or camera");
  if (p) {
    if (p->magic != kCutMagic) return fail(VY_ERR_ARG, "vy_lod_cut: prev is not a cut");
    if (p->scene != s) return fail(VY_ERR_ARG, "vy_lod_cut: prev cut belongs to another scene");
    if (p->cur < 0) return fail(VY_ERR_STATE, "vy_lod_cut: prev cut has no frontier yet");
  }
  if ((full_mode & ~(VY_CUT_FLAT | VY_CUT_DFS | VY_CUT_CHUNKED)) != 0)
    return fail(VY_ERR_ARG, "vy_lod_cut: unknown mode %d", full_mode);
  const bool chunked = (full_mode & VY_CUT_CHUNKED) != 0;
  if (chunked && (full_mode & (VY_CUT_FLAT | VY_CUT_DFS)) != 0)
    return fail(VY_ERR_ARG, "vy_lod_cut: VY_CUT_CHUNKED is a traversal of its own");
  if (chunked && !s->part)
    return fail(VY_ERR_STATE, "vy_lod_cut: VY_CUT_CHUNKED needs the scene's partition (vy_scene_partition)");
  hipStream_t st = (hipStream_t)stream;
  const LodCam L = make_cam(cam, tau);
  const uint32_t cap = (uint32_t)s->n;
  // destination frontier buffer: never the one we read from
  const int src = p ? p->cur : -1;
  const int dst = (p == o) ? 1 - src : (o->cur < 0 ? 0 : 1 - o->cur);
  const bool flat = !p && (full_mode & VY_CUT_FLAT) != 0;
  const bool dfs = (full_mode & VY_CUT_DFS) != 0;
  {
    ProfScope ps(VY_STAGE_LOD_SETUP, st);
    lod_setup<<<1, 64, 0, st>>>(o->ctr, o->q[0], (!p && !flat && !chunked) ? 1 : 0);
    VY_LAUNCHED();
  }
  if (chunked) {
    Partition* P = s->part;
    if (++P->epoch == 0) {   // the stamps would repeat: clear them (once in 2^32 searches)
      VY_HIP(hipMemsetAsync(P->stamp, 0, sizeof(uint32_t) * P->n_nodes, st));
      VY_HIP(hipMemsetAsync(P->done, 0, sizeof(uint32_t) * P->n_nodes, st));
      P->epoch = 1;
    }
    const ChunkArgs A{P->rec, P->aux, P->sub_rec, P->sub_up, P->sub_of, P->chunk_sub, P->chunk_dep, P->stamp,
                      P->done, P->ctr, P->queue[0], P->queue[1], P->n_chunks, P->n_sub};
    {
      ProfScope ps(VY_STAGE_LOD_SETUP, st);
      lod_chunk_setup<<<1, 64, 0, st>>>(P->ctr, P->stamp, P->epoch, p ? 0 : 1);
      VY_LAUNCHED();
    }
    if (!p) {
      ProfScope ps(VY_STAGE_LOD_TRAVERSE, st);
      // persistent workgroups (two fit a CU with 72 KB of LDS each)
      const int blocks = (int)(P->n_chunks < 512 ? P->n_chunks : 512);
      lod_chunk_stream<<<blocks, 256, 0, st>>>(A, L, P->epoch, o->fbits, o->cbits, o->ctr + kErr);
      VY_LAUNCHED();
    } else {
      {
        ProfScope ps(VY_STAGE_LOD_CLASSIFY, st);
        lod_sub_identify<<<2048, 256, 0, st>>>(A, p->F[src], p->counts + src, P->epoch, cap, o->ctr + kErr);
        VY_LAUNCHED();
      }
      const int blocks = (int)((P->n_sub + 255) / 256 < 2048 ? (P->n_sub + 255) / 256 : 2048);
      for (int j = 0; j < P->max_rounds; ++j) {
        ProfScope ps(VY_STAGE_LOD_TRAVERSE, st);
        lod_sub_round<<<blocks, 256, 0, st>>>(A, s->lod, L, P->epoch, j, j + 1 == P->max_rounds, o->fbits, o->cbits,
                                              o->ctr + kErr);
        VY_LAUNCHED();
      }
    }
  } else if (flat) {
    ProfScope ps(VY_STAGE_LOD_FLAT, st);
    const int64_t waves = (s->n + 63) / 64;
    const int64_t blocks = (waves + 3) / 4 < 65536 ? (waves + 3) / 4 : 65536;
    lod_flat<<<(int)blocks, 256, 0, st>>>(s->n, s->lod, L, o->fbits, o->cbits);
    VY_LAUNCHED();
  } else {
    if (p) {
      ProfScope ps(VY_STAGE_LOD_CLASSIFY, st);
      // Cut::counts[src] holds |F_prev|; if p != o the worklist of o is used (4096 workgroups:
      // 1024, 2048, 8192 and 16384 measured slower)
      lod_classify<<<4096, 256, 0, st>>>(p->F[src], p->counts + src, s->lod, s->ccount, L, o->q[0], o->ctr, cap,
                                         o->fbits, o->cbits);
      VY_LAUNCHED();
    }
    const int blocks = (int)((s->n + 255) / 256 < 1024 ? (s->n + 255) / 256 : 1024);
    if (dfs) {
      // enough level launches for the deepest possible descent
      const int launches = (s->levels + kLocalLevels - 1) / kLocalLevels;
      for (int j = 0; j < launches; ++j) {
        ProfScope ps(VY_STAGE_LOD_TRAVERSE, st);
        lod_level<kLocalLevels><<<blocks, 256, 0, st>>>(o->q[j & 1], o->ctr + kQ0, j, o->q[(j + 1) & 1], s->lod,
                                                        s->ccount, L, cap, o->fbits, o->cbits, o->ctr + kErr,
                                                        j + 1 == launches);
        VY_LAUNCHED();
      }
    } else {
      const int launches = (s->levels + kBfsLevels - 1) / kBfsLevels;
      // one subtree root per workgroup at a time: many workgroups (1024 and 2048 measured slower)
      const int bfs_blocks = (int)((s->n + 255) / 256 < 4096 ? (s->n + 255) / 256 : 4096);
      for (int j = 0; j < launches; ++j) {
        ProfScope ps(VY_STAGE_LOD_TRAVERSE, st);
        lod_bfs<<<bfs_blocks, 256, 0, st>>>(o->q[j & 1], o->ctr + kQ0, j, o->q[(j + 1) & 1], s->lod, s->ccount, L, cap,
                                        o->fbits, o->cbits, o->ctr + kErr, j + 1 == launches);
        VY_LAUNCHED();
      }
    }
  }
  {
    ProfScope ps(VY_STAGE_LOD_COMPACT, st);
    uint32_t* part_tot = reinterpret_cast<uint32_t*>(o->status);   // 2 words per partition
    lod_part_totals<<<(int)o->n_parts, 256, 0, st>>>(o->n_words, o->fbits, o->cbits, part_tot);
    VY_LAUNCHED();
    lod_compact<<<(int)o->n_parts, 256, 0, st>>>(o->n_words, o->fbits, o->cbits, o->F[dst], o->C, o->counts, dst,
                                                 part_tot, (uint32_t)o->n_parts);
    VY_LAUNCHED();
  }
  o->cur = dst;
  ++o->version;
  return VY_OK;
}

static inline int32_t bits_i(float f) {
  int32_t i;
  memcpy(&i, &f, 4);
  return i;
}
static inline float bits_f(uint32_t u) {
  float f;
  memcpy(&f, &u, 4);
  return f;
}

size_t vy_scene_partition_bytes(int64_t n) {
  if (n < 1) return 0;
  return (size_t)n * (32 + 4 * 4 + 4 + 8 + 4 * 2 + 4 * 2) + 3 * 4 * 256 + 64 * 4 + 16 * 256;
}

int vy_partition_plan(int64_t n, const int32_t* parent, const int32_t* first_child, const int32_t* child_count,
                      int32_t* sub_of, int32_t* local, int64_t* n_sub_out, int32_t* sub_root, int32_t* sub_rec,
                      int32_t* chunk_sub, int64_t* n_chunks_out) {
  if (n < 1 || !parent || !first_child || !child_count || !sub_of || !local || !n_sub_out || !sub_root ||
      !sub_rec || !chunk_sub || !n_chunks_out)
    return fail(VY_ERR_ARG, "vy_partition_plan: bad argument");
  if (parent[0] != -1) return fail(VY_ERR_ARG, "vy_partition_plan: node 0 must be the root");
  std::vector<int32_t> depth(n, 0), root_of(n, 0);
  for (int64_t i = 1; i < n; ++i) {
    const int32_t p = parent[i];
    if (p < 0 || p >= i) return fail(VY_ERR_ARG, "vy_partition_plan: parents must be numbered before children");
    depth[i] = depth[p] + 1;
  }
  // subtree roots at depths 0, 3, 6, ...; subtree ids by ascending root id (BFS order)
  int64_t n_sub = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (depth[i] % 3 == 0) {
      root_of[i] = (int32_t)i;
      sub_of[i] = (int32_t)n_sub;
      sub_root[n_sub++] = (int32_t)i;
    } else {
      root_of[i] = root_of[parent[i]];
      sub_of[i] = sub_of[root_of[i]];
    }
  }
  // nodes of each subtree in local BFS order (root, children, grandchildren)
  int64_t r = 0;
  for (int64_t s = 0; s < n_sub; ++s) {
    sub_rec[s] = (int32_t)r;
    int32_t list[kMaxSubNodes];
    int m = 0;
    list[m++] = sub_root[s];
    for (int h = 0; h < m; ++h) {
      const int32_t v = list[h];
      if (depth[v] - depth[sub_root[s]] >= 2) continue;
      for (int32_t k = 0; k < child_count[v]; ++k) {
        const int32_t c = first_child[v] + k;
        if (c <= v || c >= n || parent[c] != v) return fail(VY_ERR_ARG, "vy_partition_plan: bad child link");
        if (m >= kMaxSubNodes) return fail(VY_ERR_ARG, "vy_partition_plan: a subtree exceeds %d nodes", kMaxSubNodes);
        list[m++] = c;
      }
    }
    for (int h = 0; h < m; ++h) local[list[h]] = (int32_t)(r + h);
    r += m;
  }
  if (r != n) return fail(VY_ERR_ARG, "vy_partition_plan: the subtrees do not cover the tree");
  sub_rec[n_sub] = (int32_t)r;
  // greedy packing of consecutive subtrees into chunks of at most kChunkNodes
  // nodes: the fewest chunks under the contiguity constraint
  int64_t nc = 0, used = 0;
  for (int64_t s = 0; s < n_sub; ++s) {
    const int64_t sz = sub_rec[s + 1] - sub_rec[s];
    if (nc == 0 || used + sz > kChunkNodes) {
      chunk_sub[nc++] = (int32_t)s;
      used = 0;
    }
    used += sz;
  }
  chunk_sub[nc] = (int32_t)n_sub;
  *n_sub_out = n_sub;
  *n_chunks_out = nc;
  return VY_OK;
}

int vy_scene_partition(vy_scene* scene, void* ws, size_t bytes, void* stream) {
  Scene* s = (Scene*)scene;
  if (!s || s->magic != kSceneMagic || !ws) return fail(VY_ERR_ARG, "vy_scene_partition: bad argument");
  const int64_t n = s->n;
  if (bytes < vy_scene_partition_bytes(n))
    return fail(VY_ERR_ARG, "vy_scene_partition: workspace %zu < %zu bytes", bytes, vy_scene_partition_bytes(n));
  hipStream_t st = (hipStream_t)stream;
  std::vector<float4> lod(2 * n);
  std::vector<int32_t> cc(n);
  VY_HIP(hipMemcpyAsync(lod.data(), s->lod, sizeof(float4) * 2 * n, hipMemcpyDeviceToHost, st));
  VY_HIP(hipMemcpyAsync(cc.data(), s->ccount, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
  VY_HIP(hipStreamSynchronize(st));
  std::vector<int32_t> parent(n), fc(n), sub_of(n), local(n), sub_root(n), sub_rec(n + 1), chunk_sub(n + 1);
  for (int64_t i = 0; i < n; ++i) {
    parent[i] = bits_i(lod[2 * i + 1].w);
    fc[i] = bits_i(lod[2 * i].w);
  }
  int64_t n_sub = 0, n_chunks = 0;
  if (int rc = vy_partition_plan(n, parent.data(), fc.data(), cc.data(), sub_of.data(), local.data(), &n_sub,
                                 sub_root.data(), sub_rec.data(), chunk_sub.data(), &n_chunks))
    return rc;
  std::vector<int32_t> chunk_of(n_sub);
  for (int64_t c = 0; c < n_chunks; ++c)
    for (int32_t q = chunk_sub[c]; q < chunk_sub[c + 1]; ++q) chunk_of[q] = (int32_t)c;
  // records, subtree by subtree
  std::vector<float4> rec(2 * n);
  std::vector<int32_t> aux(n, -1), sub_up(n_sub);
  std::vector<int2> dep(n_chunks);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t k = local[i];
    const int32_t q = sub_of[i], root = sub_root[q];
    uint32_t lp = kMetaRootParent;
    if (i != root) lp = (uint32_t)(local[parent[i]] - sub_rec[q]);
    int d = 0;
    for (int32_t v = (int32_t)i; v != root; v = parent[v]) ++d;
    const bool internal = cc[i] > 0, bottom = internal && d == 2;
    const uint32_t meta = lp | (internal ? 1u << 8 : 0u) | (bottom ? 1u << 9 : 0u) |
                          ((uint32_t)(q - chunk_sub[chunk_of[q]]) << 10) |
                          ((uint32_t)(cc[i] < 2047 ? cc[i] : 2047) << 21);
    if (cc[i] > 2047) return fail(VY_ERR_ARG, "vy_scene_partition: a node has more than 2047 children");
    const float4 a = lod[2 * i], b = lod[2 * i + 1];
    rec[2 * k] = make_float4(a.x, a.y, a.z, bits_f((uint32_t)i));
    rec[2 * k + 1] = make_float4(b.x, b.y, b.z, bits_f(meta));
    if (bottom) aux[k] = sub_of[fc[i]];
  }
  int sub_levels = 1;
  for (int64_t q = 0; q < n_sub; ++q) {
    const int32_t root = sub_root[q];
    sub_up[q] = parent[root];
    if (q > 0) {
      int d = 0;
      for (int32_t v = root; v > 0; v = parent[v]) ++d;
      sub_levels = std::max(sub_levels, d / 3 + 1);
    }
  }
  for (int64_t c = 0; c < n_chunks; ++c) {
    int lo = INT32_MAX, hi = -1;
    for (int32_t q = chunk_sub[c]; q < chunk_sub[c + 1]; ++q) {
      if (sub_up[q] < 0) continue;
      const int32_t pc = chunk_of[sub_of[sub_up[q]]];
      if (pc == c) continue;
      lo = std::min(lo, pc);
      hi = std::max(hi, pc);
    }
    dep[c] = hi < 0 ? make_int2(0, -1) : make_int2(lo, hi);
  }
  Partition* P = s->part ? s->part : new (std::nothrow) Partition();
  if (!P) return fail(VY_ERR_ARG, "vy_scene_partition: out of host memory");
  Carver cv(ws, bytes);
  P->n_sub = n_sub;
  P->n_chunks = n_chunks;
  P->n_nodes = n;
  P->rec = cv.take<float4>(2 * n);
  P->aux = cv.take<int32_t>(n);
  P->sub_of = cv.take<int32_t>(n);
  P->sub_rec = cv.take<int32_t>(n + 1);
  P->sub_up = cv.take<int32_t>(n);
  P->chunk_sub = cv.take<int32_t>(n + 1);
  P->chunk_dep = cv.take<int2>(n);
  P->stamp = cv.take<uint32_t>(n);
  P->done = cv.take<uint32_t>(n);
  P->queue[0] = cv.take<int32_t>(n);
  P->queue[1] = cv.take<int32_t>(n);
  P->ctr = cv.take<uint32_t>(64);
  P->epoch = 0;
  P->max_rounds = 2 * sub_levels + 2;
  int rc = VY_OK;
  if (!cv.ok()) rc = fail(VY_ERR_ARG, "vy_scene_partition: workspace layout overflow");
  hipError_t e = hipSuccess;
  if (rc == VY_OK) {
    e = hipMemcpyAsync(P->rec, rec.data(), sizeof(float4) * 2 * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(P->aux, aux.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(P->sub_of, sub_of.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(P->sub_rec, sub_rec.data(), sizeof(int32_t) * (n_sub + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(P->sub_up, sub_up.data(), sizeof(int32_t) * n_sub, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(P->chunk_sub, chunk_sub.data(), sizeof(int32_t) * (n_chunks + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(P->chunk_dep, dep.data(), sizeof(int2) * n_chunks, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(P->stamp, 0, sizeof(uint32_t) * n, st);
    if (e == hipSuccess) e = hipMemsetAsync(P->done, 0, sizeof(uint32_t) * n, st);
    if (e == hipSuccess) e = hipMemsetAsync(P->ctr, 0, 64 * 4, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = fail(VY_ERR_HIP, "vy_scene_partition: %s", hipGetErrorString(e));
  }
  if (rc != VY_OK) {
    if (!s->part) delete P;
    return rc;
  }
  s->part = P;
  return VY_OK;
}

int vy_cut_counts(const vy_cut* cut, int64_t* n_frontier, int64_t* n_cut, void* stream) {
  const Cut* c = (const Cut*)cut;
  if (!c || c->magic != kCutMagic) return fail(VY_ERR_ARG, "vy_cut_counts: bad argument");
  if (c->cur < 0) return fail(VY_ERR_STATE, "vy_cut_counts: no cut computed yet");
  int32_t h[4];
  uint32_t e[4];
  hipStream_t st = (hipStream_t)stream;
  VY_HIP(hipMemcpyAsync(h, c->counts, sizeof(h), hipMemcpyDeviceToHost, st));
  VY_HIP(hipMemcpyAsync(e, c->ctr, sizeof(e), hipMemcpyDeviceToHost, st));
  VY_HIP(hipStreamSynchronize(st));
  if (n_frontier) *n_frontier = h[c->cur];
  if (n_cut) *n_cut = h[2];
  if (e[kErr]) return fail(VY_ERR_DEVICE, "vy_lod_cut: device-side bound hit (%u)", e[kErr]);
  return VY_OK;
}

int vy_cut_arrays(const vy_cut* cut, const int32_t** frontier, const int32_t** cut_ids, const int32_t** counts) {
  const Cut* c = (const Cut*)cut;
  if (!c || c->magic != kCutMagic) return fail(VY_ERR_ARG, "vy_cut_arrays: bad argument");
  if (c->cur < 0) return fail(VY_ERR_STATE, "vy_cut_arrays: no cut computed yet");
  if (frontier) *frontier = c->F[c->cur];
  if (cut_ids) *cut_ids = c->C;
  if (counts) *counts = c->counts;
  return VY_OK;
}

int vy_cut_set_frontier(vy_cut* cut, const int32_t* ids, int64_t n, void* stream) {
  Cut* c = (Cut*)cut;
  if (!c || c->magic != kCutMagic || (!ids && n > 0)) return fail(VY_ERR_ARG, "vy_cut_set_frontier: bad argument");
  if (n < 1 || n > c->n) return fail(VY_ERR_ARG, "vy_cut_set_frontier: n %lld out of range", (long long)n);
  hipStream_t st = (hipStream_t)stream;
  const int dst = c->cur < 0 ? 0 : 1 - c->cur;
  VY_HIP(hipMemcpyAsync(c->F[dst], ids, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
  set_count<<<1, 64, 0, st>>>(c->counts + dst, (int32_t)n);
  VY_LAUNCHED();
  c->cur = dst;
  ++c->version;
  return VY_OK;
}

}  // extern "C"

// Accessors for the render stage (same library).
namespace vy {
const int32_t* cut_ids_dev(const Cut* c) { return c->C; }
const int32_t* cut_count_dev(const Cut* c) { return c->counts + 2; }
const int32_t* cut_frontier_count_dev(const Cut* c) { return c->counts + (c->cur < 0 ? 0 : c->cur); }
const uint32_t* cut_err_dev(const Cut* c) { return c->ctr + kErr; }
}  // namespace vy
