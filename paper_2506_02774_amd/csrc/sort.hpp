// Stable LSD radix sort passes (onesweep: one scatter launch per digit with
// decoupled look-back across partitions) for uint32 keys and uint32 values on
// gfx950 (wave64, LDS staging).
//
// Included by render.hip only.
#pragma once

#include "vy_common.hpp"

namespace vysort {

using namespace vyd;

// 1024-thread workgroups of 16 waves, 12 keys per thread: 12288 keys per
// partition, so that a pass over a few million keys needs a few hundred
// partitions (a short look-back chain) that all run at once. (8 and 16 keys
// per thread were measured slower: a longer chain, and one workgroup per CU
// with too little LDS left, respectively.)
constexpr int kThreads = 1024;
constexpr int kItems = 12;                    // keys per thread per partition
constexpr int kTile = kThreads * kItems;      // keys per partition
constexpr int kWaves = kThreads / 64;
constexpr int kLookback = 4;                  // predecessors polled per step of a digit's look-back

// Exclusive scan of one value per thread of the first 256 threads of the
// block (all threads call it; the others pass 0 and get 0). `sh` needs 5 words.
VY_DEV uint32_t scan_first256(uint32_t v, uint32_t* sh, uint32_t* total) {
  const uint32_t l = lane(), w = threadIdx.x >> 6;
  uint32_t x = w < 4 ? v : 0u;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (l >= (uint32_t)o) x += y;
  }
  if (w < 4 && l == 63) sh[w] = x;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t s = sh[i];
    if (i < (int)w) wbase += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return w < 4 ? wbase + x - v : 0u;
}

// One stable scatter pass on digit (key >> shift) & mask (mask <= 255).
// `ghist` holds this digit's global histogram (256 counts of the n keys).
// vals_in == nullptr means value = input index. n = min(*n_ptr, n_cap).
// Partitions are taken in ticket order; each publishes its 256 digit counts
// and looks back for its predecessors' (`status`, 256 words per partition).
__global__ __launch_bounds__(kThreads) void onesweep_pass(const uint32_t* __restrict__ keys_in,
                                                          const uint32_t* __restrict__ vals_in,
                                                          uint32_t* __restrict__ keys_out,
                                                          uint32_t* __restrict__ vals_out, const uint32_t* n_ptr,
                                                          uint32_t n_cap, int shift, uint32_t mask, int nbits,
                                                          const uint32_t* __restrict__ ghist, uint64_t* status,
                                                          uint32_t epoch, uint32_t* ticket, uint32_t* err) {
  __shared__ uint32_t s_keys[kTile];
  __shared__ uint32_t s_vals[kTile];
  __shared__ uint32_t s_whist[kWaves][256];
  __shared__ uint32_t s_dstart[256];
  __shared__ uint32_t s_gofs[256];
  __shared__ uint32_t s_gstart[256];
  __shared__ uint32_t s_scan[8];
  __shared__ uint32_t s_part;

  const uint32_t tid = threadIdx.x, w = tid >> 6, l = lane();
  uint32_t n = *n_ptr;
  if (n > n_cap) n = n_cap;
  const uint32_t n_parts = (n + kTile - 1) / kTile;
  {
    uint32_t tot;
    const uint32_t g = tid < 256 ? ghist[tid] : 0u;
    const uint32_t x = scan_first256(g, s_scan, &tot);
    if (tid < 256) s_gstart[tid] = x;
  }
  for (;;) {
    if (tid == 0) s_part = fetch_add(ticket, 1u);
    s_whist[w][l] = 0;
    s_whist[w][l + 64] = 0;
    s_whist[w][l + 128] = 0;
    s_whist[w][l + 192] = 0;
    __syncthreads();
    const uint32_t part = s_part;
    if (part >= n_parts) break;
    const uint32_t base = part * kTile;
    const uint32_t cnt = (n - base) < (uint32_t)kTile ? (n - base) : (uint32_t)kTile;
    uint32_t key[kItems], val[kItems], rnk[kItems];
    // load: wave w round r covers partition items w*64*kItems + r*64 + lane (ranking order)
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t li = w * (64 * kItems) + r * 64 + l;
      const bool ok = li < cnt;
      key[r] = ok ? keys_in[base + li] : 0xFFFFFFFFu;
      val[r] = ok ? (vals_in ? vals_in[base + li] : base + li) : 0u;
    }
    // rank within the wave: lanes with the same digit found by ballots over
    // its bits, counted in order against the wave's running digit counts
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t li = w * (64 * kItems) + r * 64 + l;
      const bool ok = li < cnt;
      const uint32_t d = (key[r] >> shift) & mask;
      uint64_t peers = ballot(ok);
      for (int b = 0; b < nbits; ++b) {
        const uint64_t bb = ballot(((d >> b) & 1u) != 0);
        peers &= ((d >> b) & 1u) ? bb : ~bb;
      }
      const uint32_t before = s_whist[w][d];
      const uint32_t rk = (uint32_t)__popcll(peers & lanemask_lt());
      rnk[r] = before + rk;
      const bool leader = ok && rk == 0;
      // all lanes read the running count before the leader updates it (same wave, in order)
      __builtin_amdgcn_wave_barrier();
      if (leader) s_whist[w][d] = before + (uint32_t)__popcll(peers);
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit: wave exclusive offsets and the partition total
    uint32_t dtot = 0;
    if (tid < 256) {
      uint32_t run = 0;
#pragma unroll
      for (int ww = 0; ww < kWaves; ++ww) {
        const uint32_t c = s_whist[ww][tid];
        s_whist[ww][tid] = run;
        run += c;
      }
      dtot = run;
    }
    // the partition's digit counts go out before anything else, so that
    // successors looking back are held up as little as possible
    if (tid < 256) publish_aggregate(status + tid, part, 256, epoch, dtot);
    uint32_t btot;
    const uint32_t dstart = scan_first256(dtot, s_scan, &btot);
    if (tid < 256) s_dstart[tid] = dstart;
    __syncthreads();
    // local scatter into digit order first: the keys leave the registers
    // before the look-back, which then polls kLookback predecessors per step
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t li = w * (64 * kItems) + r * 64 + l;
      if (li < cnt) {
        const uint32_t d = (key[r] >> shift) & mask;
        const uint32_t pos = s_dstart[d] + s_whist[w][d] + rnk[r];
        s_keys[pos] = key[r];
        s_vals[pos] = val[r];
      }
    }
    if (tid < 256) {
      const uint64_t ex = lookback_poll<kLookback>(status + tid, part, 256, epoch, dtot, err);
      s_gofs[tid] = s_gstart[tid] + (uint32_t)ex - dstart;
    }
    __syncthreads();
    for (uint32_t i = tid; i < cnt; i += kThreads) {
      const uint32_t k = s_keys[i];
      const uint32_t d = (k >> shift) & mask;
      const uint32_t o = s_gofs[d] + i;
      if (o < n) {   // always true unless a look-back wait timed out
        keys_out[o] = k;
        vals_out[o] = s_vals[i];
      }
    }
    __syncthreads();
  }
}

}  // namespace vysort
