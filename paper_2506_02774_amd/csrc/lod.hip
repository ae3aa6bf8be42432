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
#include <cstdlib>
#include <cstring>

#include "vy_common.hpp"

#pragma clang fp contract(off)

namespace {

using namespace vyd;

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
// 1024 words, zeroing the bitmaps as they are read: a first launch counts
// every partition's bits, and each partition of the second sums the counts
// of the partitions before it (at most a few thousand words, read from L2)
// instead of waiting on a look-back chain across the partitions.
// A partition is read as 4 rounds of 256 consecutive words (one per thread);
// each round's ids are gathered in LDS and written out with coalesced stores.
// The 8 per-thread counts (2 bitmaps x 4 rounds, each <= 32) are scanned in
// one pass as 16-bit fields of 4 words (a partition's totals stay below 2^16).
constexpr int kWordsPerThread = 4, kWordsPerPart = 256 * kWordsPerThread;

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
  __shared__ int32_t s_ids[256 * 32];
  const uint32_t part = blockIdx.x;
  if (threadIdx.x < 2) s_ex[threadIdx.x] = 0u;
  __syncthreads();
  {
    // the offsets of this partition's ids: totals of the partitions before it
    uint32_t pa = 0u, pb = 0u;
    for (uint32_t j = threadIdx.x; j < part; j += 256) {
      pa += part_tot[2 * (size_t)j];
      pb += part_tot[2 * (size_t)j + 1];
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
  const int64_t base = (int64_t)part * kWordsPerPart;
  uint32_t wd[2][kWordsPerThread];
#pragma unroll
  for (int k = 0; k < kWordsPerThread; ++k) {
    const int64_t w = base + k * 256 + threadIdx.x;
    wd[0][k] = w < n_words ? fbits[w] : 0u;
    wd[1][k] = w < n_words ? cbits[w] : 0u;
  }
  // fields: .x = F rounds 0 | 1 << 16, .y = F rounds 2 | 3, .z/.w the same for C
  const uint4 cnt4 = make_uint4((uint32_t)__popc(wd[0][0]) | ((uint32_t)__popc(wd[0][1]) << 16),
                                (uint32_t)__popc(wd[0][2]) | ((uint32_t)__popc(wd[0][3]) << 16),
                                (uint32_t)__popc(wd[1][0]) | ((uint32_t)__popc(wd[1][1]) << 16),
                                (uint32_t)__popc(wd[1][2]) | ((uint32_t)__popc(wd[1][3]) << 16));
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
      tot[q] = rt[q][0] + rt[q][1] + rt[q][2] + rt[q][3];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    int32_t* out = (q == 0 ? Fout : Cout) + s_ex[q];
    uint32_t r0 = 0;   // ids of the partition before this round
#pragma unroll
    for (int k = 0; k < kWordsPerThread; ++k) {
      const int64_t w = base + k * 256 + threadIdx.x;
      uint32_t m = wd[q][k], o = off[q][k];
      while (m) {
        const int b = __ffs(m) - 1;
        m &= m - 1;
        s_ids[o++] = (int32_t)(w * 32 + b);
      }
      __syncthreads();
      for (uint32_t i = threadIdx.x; i < rt[q][k]; i += 256) out[r0 + i] = s_ids[i];
      r0 += rt[q][k];
      if (wd[q][k]) (q == 0 ? fbits : cbits)[w] = 0u;
      __syncthreads();
    }
  }
  if (part == n_parts - 1 && threadIdx.x == 0) {
    counts[f_slot] = (int32_t)(s_ex[0] + tot[0]);
    counts[2] = (int32_t)(s_ex[1] + tot[1]);
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
  if ((full_mode & ~(VY_CUT_FLAT | VY_CUT_DFS)) != 0)
    return fail(VY_ERR_ARG, "vy_lod_cut: unknown mode %d", full_mode);
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
    lod_setup<<<1, 64, 0, st>>>(o->ctr, o->q[0], (!p && !flat) ? 1 : 0);
    VY_LAUNCHED();
  }
  if (flat) {
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
