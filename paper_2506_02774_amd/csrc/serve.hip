// Multi-viewer serving runtime: a first-fit arena over caller-owned device
// memory, admission of viewer sessions, and a host dispatch loop that issues
// their frames (vy_lod_cut + vy_render) on several HIP streams.
//
// The admission and scheduling policy is written once (Runner) over an
// executor: HipExec enqueues real frames and reads HIP events; SimExec models
// each frame as a fixed busy time on its stream in virtual time, so the same
// policy can be exercised and checked without a GPU (vy_server_simulate).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <new>
#include <set>
#include <thread>
#include <vector>

#include "vy_common.hpp"
#include "../../include/vy_serve.h"

using namespace vy;

namespace {

constexpr uint32_t kArenaMagic = 0x5659414Eu, kServerMagic = 0x56595356u;
constexpr size_t kGranule = 256;

inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ------------------------------------------------------------------ arena ----

struct Arena {
  uint32_t magic = kArenaMagic;
  uintptr_t base = 0;
  size_t bytes = 0;
  std::map<size_t, size_t> free_blocks;  // offset -> size; address order; never adjacent
  std::map<size_t, size_t> live;         // offset -> size
  size_t used = 0;

  size_t largest() const {
    size_t m = 0;
    for (const auto& f : free_blocks) m = std::max(m, f.second);
    return m;
  }
  int alloc(size_t want, void** out) {
    *out = nullptr;
    if (want == 0) return fail(VY_ERR_ARG, "vy_arena_alloc: zero bytes");
    if (want > bytes) return fail(VY_ERR_CAPACITY, "vy_arena_alloc: %zu bytes exceed the arena (%zu)", want, bytes);
    const size_t need = round_up(want, kGranule);
    for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
      if (it->second < need) continue;
      const size_t off = it->first, sz = it->second;
      free_blocks.erase(it);
      if (sz > need) free_blocks.emplace(off + need, sz - need);
      live.emplace(off, need);
      used += need;
      *out = (void*)(base + off);
      return VY_OK;
    }
    return fail(VY_ERR_CAPACITY, "vy_arena_alloc: no free block of %zu bytes (largest %zu)", need, largest());
  }
  int release(void* p) {
    const uintptr_t a = (uintptr_t)p;
    auto it = a >= base ? live.find(a - base) : live.end();
    if (it == live.end()) return fail(VY_ERR_ARG, "vy_arena_release: %p does not start a live block", p);
    size_t off = it->first, sz = it->second;
    live.erase(it);
    used -= sz;
    auto nx = free_blocks.lower_bound(off);
    if (nx != free_blocks.end() && off + sz == nx->first) {
      sz += nx->second;
      nx = free_blocks.erase(nx);
    }
    if (nx != free_blocks.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        pv->second += sz;
        return VY_OK;
      }
    }
    free_blocks.emplace(off, sz);
    return VY_OK;
  }
};

Arena* as_arena(const vy_arena* a) {
  Arena* r = (Arena*)a;
  return r && r->magic == kArenaMagic ? r : nullptr;
}

// -------------------------------------------------------------- sessions ----

// A resident session holds two arena blocks: its cut workspace and image
// (fixed size) and its render workspace, which grows when a frame overflows
// a capacity the caller left to the runtime.
struct SessionPlan {
  int64_t n_nodes = 0, max_g = 0, max_pairs = 0;
  bool grow_g = false, grow_pairs = false;   // capacities chosen by the runtime
  size_t cut_bytes = 0, image_bytes = 0, fixed = 0, render_bytes = 0, total = 0;
};

constexpr int64_t kMaxPairsCap = 0x7FFFFFFF;

// Served frames never split tiles: their contexts leave out those buffers.
size_t render_bytes_for(const vy_session* s, int64_t max_g, int64_t max_pairs) {
  return round_up(render_workspace_bytes(max_g, s->width, s->height, max_pairs, false), kGranule);
}

// `batched`: frames are rendered in batches (vy_render_batch) with the
// stream's batch context, so the session holds no render workspace and its
// capacities are the batch's.
bool plan_session(const vy_session* s, SessionPlan* p, bool batched = false) {
  if (!s) return false;
  const Scene* sc = (const Scene*)s->scene;
  if (!sc || sc->magic != kSceneMagic) return false;
  if (s->width < 1 || s->height < 1 || s->width > 32768 || s->height > 32768) return false;
  if (!(s->tau >= 0.f) || !std::isfinite(s->tau) || s->max_gaussians < 0 || s->max_pairs < 0 ||
      s->max_pairs > kMaxPairsCap)
    return false;
  const int64_t px = (int64_t)s->width * s->height;
  p->n_nodes = sc->n;
  p->grow_g = s->max_gaussians == 0;
  p->grow_pairs = s->max_pairs == 0;
  p->max_g = p->grow_g ? std::min<int64_t>(sc->n, 2 * px) : s->max_gaussians;
  p->max_pairs = p->grow_pairs ? std::min<int64_t>(4 * px, kMaxPairsCap) : s->max_pairs;
  p->cut_bytes = round_up(vy_cut_workspace_bytes(sc->n), kGranule);
  p->image_bytes = round_up((size_t)px * 3 * sizeof(float), kGranule);
  p->fixed = p->cut_bytes + p->image_bytes;
  p->render_bytes = batched ? 0 : render_bytes_for(s, p->max_g, p->max_pairs);
  if (batched) p->grow_g = p->grow_pairs = false;
  if (!p->cut_bytes || (!batched && !p->render_bytes)) return false;
  p->total = p->fixed + p->render_bytes;
  return true;
}

// --------------------------------------------------------------- policy ----

struct Resident {
  int session = -1;
  void* mem = nullptr;    // cut workspace + image
  void* rmem = nullptr;   // render workspace
  int64_t cap_g = 0, cap_pairs = 0;
  int stream = -1;
  int inflight = 0;
  int64_t left = 0;       // frames not finished yet
  double t_admit = 0;
  // growth: capacity needed by overflowed frames, and those frames
  bool grow = false;
  int64_t need_g = 0, need_pairs = 0;
  std::vector<int64_t> redo;
  // GPU state (HipExec)
  vy_cut* cut = nullptr;
  vy_render_ctx* ctx = nullptr;
  bool has_cut = false;
};

struct Ticket {
  int64_t req = -1;
  int slot = -1;
  hipEvent_t start = nullptr, done = nullptr;  // HipExec
  double t_start = 0, t_done = 0;              // SimExec
};

// What a finished frame reports back to the policy.
struct Outcome {
  double t_start = 0, t_done = 0;
  uint32_t flags = 0, n_cut = 0, n_pairs = 0;
};

struct RunCounters {
  int64_t admitted = 0, waited = 0, peak_resident = 0;
  size_t peak_bytes = 0;
  int64_t regrown = 0, redone = 0;
};

constexpr uint32_t kFlagPairs = 1, kFlagCut = 2;

// Admission (first come, first served under a slot limit and the arena),
// oldest-request-first dispatch with stream affinity while a session has
// unfinished frames, completion in stream order, and growth of the render
// workspace of a session whose frame overflowed a runtime-chosen capacity
// (the session pauses until its frames have drained, its render block is
// replaced by a larger one, and the overflowed frames are rendered again).
template <class Exec>
struct Runner {
  Exec& ex;
  Arena* arena;
  int n_streams, max_inflight, max_viewers;
  const vy_frame_req* reqs;
  int64_t n_reqs;
  int32_t n_sessions;
  const SessionPlan* plans;
  bool realtime;
  vy_frame_result* results;
  RunCounters cnt;

  std::vector<int> slot_of;                    // per session: resident slot or -1
  std::vector<int64_t> total;                  // frames per session
  std::vector<std::deque<int64_t>> waitq;      // released, not yet dispatched
  std::vector<char> in_pending, blocked;
  std::deque<int> pending;
  std::vector<Resident> res;
  std::vector<int> free_slots;
  std::vector<std::deque<Ticket>> fl;          // per stream, in enqueue order
  int resident = 0;
  int64_t n_done = 0;

  Runner(Exec& e, Arena* a, int ns, int mi, int mv, const vy_frame_req* r, int64_t nr, int32_t nsess,
         const SessionPlan* p, bool rt, vy_frame_result* out)
      : ex(e), arena(a), n_streams(ns), max_inflight(mi), max_viewers(mv), reqs(r), n_reqs(nr), n_sessions(nsess),
        plans(p), realtime(rt), results(out) {}

  void release(int slot) {
    Resident& r = res[slot];
    ex.release(r);
    (void)arena->release(r.mem);
    if (r.rmem) (void)arena->release(r.rmem);
    slot_of[r.session] = -1;
    r = Resident();
    free_slots.push_back(slot);
    --resident;
  }

  int abandon(int rc) {
    ex.drain();
    for (auto& q : fl)
      for (auto& t : q) ex.recycle(t);
    for (int s = 0; s < (int)res.size(); ++s)
      if (res[s].session >= 0) release(s);
    return rc;
  }

  void note_peak() {
    cnt.peak_resident = std::max<int64_t>(cnt.peak_resident, resident);
    cnt.peak_bytes = std::max(cnt.peak_bytes, arena->used);
  }

  // A finished frame: final (true), or queued again after its session grows.
  bool finish(int slot, int64_t req, const Outcome& o) {
    Resident& r = res[slot];
    const SessionPlan& p = plans[r.session];
    --r.inflight;
    const bool g = (o.flags & kFlagCut) && p.grow_g && r.cap_g < p.n_nodes;
    const bool q = (o.flags & kFlagPairs) && p.grow_pairs && r.cap_pairs < kMaxPairsCap;
    results[req].t_start = o.t_start;
    results[req].t_done = o.t_done;
    if (g || q) {
      r.grow = true;
      if (g) r.need_g = std::max<int64_t>(r.need_g, o.n_cut);
      if (q) r.need_pairs = std::max<int64_t>(r.need_pairs, o.n_pairs);
      r.redo.push_back(req);
      ++cnt.redone;
      return false;
    }
    if (--r.left == 0) release(slot);
    return true;
  }

  // Replaces the render block of a paused session once its frames drained.
  bool try_grow(int slot) {
    Resident& r = res[slot];
    const SessionPlan& p = plans[r.session];
    int64_t g = r.cap_g, q = r.cap_pairs;
    if (r.need_g > 0) g = std::min<int64_t>(p.n_nodes, std::max<int64_t>(2 * r.cap_g, r.need_g + r.need_g / 4));
    if (r.need_pairs > 0)
      q = std::min<int64_t>(kMaxPairsCap, std::max<int64_t>(2 * r.cap_pairs, r.need_pairs + r.need_pairs / 4));
    void* mem = nullptr;
    const size_t want = ex.render_bytes(r.session, g, q);
    // no frame of the session is in flight: its render block goes back first,
    // so that the larger one may take its place
    const size_t had = r.rmem ? ex.render_bytes(r.session, r.cap_g, r.cap_pairs) : 0;
    ex.drop_render(r);
    if (r.rmem) (void)arena->release(r.rmem);
    r.rmem = nullptr;
    if (arena->alloc(want, &mem) != VY_OK) {
      // the old size fits again: the block just released (merged with free
      // neighbours) holds it
      if (had && arena->alloc(had, &r.rmem) != VY_OK) return false;
      // wait while another resident session can still run and give memory back
      bool others_run = false;
      for (int o = 0; o < max_viewers; ++o)
        if (o != slot && res[o].session >= 0 && (!res[o].grow || res[o].inflight > 0)) others_run = true;
      if (others_run && want + p.fixed <= arena->bytes) return false;
      // never fits (larger than the arena, or every other resident session is
      // itself paused for memory): keep the frames as they are (flagged)
      r.grow = false;
      r.need_g = r.need_pairs = 0;
      n_done += (int64_t)r.redo.size();
      r.left -= (int64_t)r.redo.size();
      r.redo.clear();
      if (r.left == 0) release(slot);
      return true;
    }
    r.rmem = mem;
    r.cap_g = g;
    r.cap_pairs = q;
    r.grow = false;
    r.need_g = r.need_pairs = 0;
    std::sort(r.redo.begin(), r.redo.end());
    auto& w = waitq[r.session];
    for (auto it = r.redo.rbegin(); it != r.redo.rend(); ++it) w.push_front(*it);
    r.redo.clear();
    ++cnt.regrown;
    note_peak();
    return true;
  }

  int run() {
    slot_of.assign(n_sessions, -1);
    total.assign(n_sessions, 0);
    waitq.assign(n_sessions, {});
    in_pending.assign(n_sessions, 0);
    blocked.assign(n_sessions, 0);
    res.assign(max_viewers, Resident());
    free_slots.clear();
    for (int s = max_viewers - 1; s >= 0; --s) free_slots.push_back(s);
    fl.assign(n_streams, {});
    for (int64_t i = 0; i < n_reqs; ++i) ++total[reqs[i].session];
    int64_t next_rel = 0;
    n_done = 0;
    while (n_done < n_reqs) {
      bool progress = false;
      const double now = ex.now();
      // 1. release arrived requests
      while (next_rel < n_reqs && (!realtime || reqs[next_rel].t_arrival <= now)) {
        const int s = reqs[next_rel].session;
        waitq[s].push_back(next_rel);
        if (slot_of[s] < 0 && !in_pending[s]) {
          pending.push_back(s);
          in_pending[s] = 1;
        }
        ++next_rel;
        progress = true;
      }
      // 2. retire finished frames, stream by stream in enqueue order
      for (int k = 0; k < n_streams; ++k) {
        while (!fl[k].empty()) {
          Ticket& t = fl[k].front();
          Outcome o;
          const int q = ex.poll(t, &o);
          if (q < 0) return abandon(q);
          if (q == 0) break;
          const int slot = t.slot;
          const int64_t req = t.req;
          ex.recycle(t);
          fl[k].pop_front();
          if (finish(slot, req, o)) ++n_done;
          progress = true;
        }
      }
      // 3. grow paused sessions whose frames have drained
      for (int slot = 0; slot < max_viewers; ++slot)
        if (res[slot].session >= 0 && res[slot].grow && res[slot].inflight == 0 && try_grow(slot)) progress = true;
      if (n_done == n_reqs) break;
      // 4. admit waiting sessions in arrival order
      while (!pending.empty()) {
        const int s = pending.front();
        const SessionPlan& p = plans[s];
        void* mem = nullptr;
        void* rmem = nullptr;
        if (free_slots.empty() || arena->alloc(p.fixed, &mem) != VY_OK) {
          blocked[s] = 1;
          break;
        }
        if (p.render_bytes > 0 && arena->alloc(p.render_bytes, &rmem) != VY_OK) {
          (void)arena->release(mem);
          blocked[s] = 1;
          break;
        }
        pending.pop_front();
        in_pending[s] = 0;
        const int slot = free_slots.back();
        free_slots.pop_back();
        Resident& r = res[slot];
        r = Resident();
        r.session = s;
        r.mem = mem;
        r.rmem = rmem;
        r.cap_g = p.max_g;
        r.cap_pairs = p.max_pairs;
        r.left = total[s];
        r.t_admit = now;
        slot_of[s] = slot;
        ++resident;
        ++cnt.admitted;
        cnt.waited += blocked[s] ? 1 : 0;
        note_peak();
        progress = true;
      }
      // 5. dispatch: oldest released request of a resident session whose stream has room
      for (;;) {
        int best_slot = -1, best_stream = -1;
        int64_t best_req = INT64_MAX;
        int least = -1;
        for (int k = 0; k < n_streams; ++k)
          if ((int)fl[k].size() < max_inflight && (least < 0 || fl[k].size() < fl[least].size())) least = k;
        for (int slot = 0; slot < max_viewers; ++slot) {
          const Resident& r = res[slot];
          if (r.session < 0 || r.grow || waitq[r.session].empty()) continue;
          const int k = r.inflight > 0 ? r.stream : least;
          if (k < 0 || (int)fl[k].size() >= max_inflight || !ex.can_take(r, k)) continue;
          const int64_t q = waitq[r.session].front();
          if (q < best_req) {
            best_req = q;
            best_slot = slot;
            best_stream = k;
          }
        }
        if (best_slot < 0) break;
        Resident& r = res[best_slot];
        waitq[r.session].pop_front();
        vy_frame_result& out = results[best_req];
        out.t_admit = r.t_admit;
        out.t_dispatch = ex.now();
        out.stream = best_stream;
        Ticket t;
        t.req = best_req;
        t.slot = best_slot;
        int32_t status = VY_OK;
        const int rc = ex.dispatch(r, best_req, best_stream, &t, &status);
        if (rc != VY_OK) {
          ex.recycle(t);
          return abandon(rc);
        }
        out.status = status;
        r.stream = best_stream;
        ++r.inflight;
        fl[best_stream].push_back(t);
        progress = true;
      }
      // 6. enqueue what the executor gathered (batched frames)
      if (int rc = ex.flush()) return abandon(rc);
      if (n_done == n_reqs) break;
      if (!progress) {
        const double next = next_rel < n_reqs && realtime ? reqs[next_rel].t_arrival : INFINITY;
        int64_t inflight = 0;
        for (const auto& q : fl) inflight += (int64_t)q.size();
        const int rc = ex.wait(next, inflight);
        if (rc != VY_OK) return abandon(rc);
      }
    }
    return VY_OK;
  }
};

// ------------------------------------------------------------ executors ----

double host_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct HipExec {
  const vy_session* sessions;
  const SessionPlan* plans;
  const vy_frame_req* reqs;
  vy_frame_stats* stats;        // device records (the caller's, or a block of the arena)
  vy_frame_stats* host_stats;   // pinned host copies, read when a frame has finished
  hipStream_t* streams;
  int n_streams;
  std::vector<hipEvent_t>* pool;
  hipEvent_t t0_event;
  double t0 = 0;

  double now() const { return host_seconds() - t0; }
  size_t render_bytes(int s, int64_t g, int64_t q) const { return render_bytes_for(&sessions[s], g, q); }

  int dispatch(Resident& r, int64_t i, int k, Ticket* t, int32_t* status) {
    const vy_frame_req& q = reqs[i];
    const vy_session& ss = sessions[r.session];
    const SessionPlan& p = plans[r.session];
    hipStream_t st = streams[k];
    char* mem = (char*)r.mem;
    // handles over the session's arena blocks, initialised on this stream
    if (!r.cut && cut_create_on(ss.scene, mem, p.cut_bytes, st, false, &r.cut) != VY_OK) return VY_ERR_HIP;
    if (!r.ctx && render_ctx_create_on(r.cap_g, ss.width, ss.height, r.cap_pairs, false, r.rmem,
                                       render_bytes_for(&ss, r.cap_g, r.cap_pairs), st, false, &r.ctx) != VY_OK)
      return VY_ERR_HIP;
    if (pool->size() < 2) return fail(VY_ERR_HIP, "vy_server_run: event pool exhausted");
    t->start = pool->back();
    pool->pop_back();
    t->done = pool->back();
    pool->pop_back();
    VY_HIP(hipEventRecord(t->start, st));
    float* image = q.image ? q.image : (float*)(mem + p.cut_bytes);
    // the record may hold an earlier attempt of this frame: the hash is summed into it
    VY_HIP(hipMemsetAsync(stats + i, 0, sizeof(vy_frame_stats), st));
    int rc = vy_lod_cut(ss.scene, &q.cam, ss.tau, r.has_cut ? r.cut : nullptr, r.cut, VY_CUT_FRONTIER, st);
    if (rc == VY_OK) {
      r.has_cut = true;
      vy_render_opts o;
      memset(&o, 0, sizeof(o));
      o.alpha_filter = ss.alpha_filter;
      if (n_streams > 1) o.band_jobs = 2;   // frames of several streams overlap: the throughput layout
      rc = vy_render(ss.scene, r.cut, &q.cam, &o, image, r.ctx, st);
    }
    if (rc == VY_OK) rc = render_frame_finish(r.cut, r.ctx, image, ss.width, ss.height, stats + i, st);
    if (rc == VY_ERR_HIP) return rc;
    *status = rc;
    VY_HIP(hipMemcpyAsync(host_stats + i, stats + i, sizeof(vy_frame_stats), hipMemcpyDeviceToHost, st));
    VY_HIP(hipEventRecord(t->done, st));
    return VY_OK;
  }

  int poll(const Ticket& t, Outcome* o) {
    const hipError_t e = hipEventQuery(t.done);
    if (e == hipErrorNotReady) return 0;
    if (e != hipSuccess) return fail(VY_ERR_HIP, "vy_server_run: hipEventQuery: %s", hipGetErrorString(e));
    float a = 0, b = 0;
    VY_HIP(hipEventElapsedTime(&a, t0_event, t.start));
    VY_HIP(hipEventElapsedTime(&b, t0_event, t.done));
    o->t_start = a * 1e-3;
    o->t_done = b * 1e-3;
    const vy_frame_stats& h = host_stats[t.req];
    o->flags = h.flags;
    o->n_cut = h.n_cut;
    o->n_pairs = h.n_pairs;
    return 1;
  }

  void recycle(Ticket& t) {
    if (t.start) pool->push_back(t.start);
    if (t.done) pool->push_back(t.done);
    t.start = t.done = nullptr;
  }

  void drop_render(Resident& r) {
    if (r.ctx) vy_render_ctx_free(r.ctx);
    r.ctx = nullptr;
  }

  void release(Resident& r) {
    if (r.cut) vy_cut_free(r.cut);
    drop_render(r);
    r.cut = nullptr;
  }

  int wait(double next_arrival, int64_t inflight) {
    // nothing to do until a frame finishes (poll) or the next request arrives (sleep)
    if (inflight == 0 && !std::isfinite(next_arrival))
      return fail(VY_ERR_STATE, "vy_server_run: nothing in flight and no request to wait for");
    const double gap = next_arrival - now();
    if (inflight == 0 && gap > 300e-6)
      std::this_thread::sleep_for(std::chrono::microseconds((int64_t)((gap - 200e-6) * 1e6)));
    else
      std::this_thread::yield();
    return VY_OK;
  }

  void drain() {
    for (int k = 0; k < n_streams; ++k) (void)hipStreamSynchronize(streams[k]);
  }

  bool can_take(const Resident&, int) const { return true; }
  int flush() { return VY_OK; }
};

// Batched frames: dispatch gathers frames per stream (one per session, one
// alpha_filter, at most max_batch frames and VY_BATCH_MAX_TILES tiles), and a
// gathered batch is enqueued on its stream when it is full or when the
// stream's previous batch has finished (so that one batch runs while the next
// one gathers the frames that arrive or become ready meanwhile): the frames'
// searches (vy_lod_cut, each from its session's previous frontier), one
// vy_render_batch with the stream's batch context, and the frames' records.
// A frame's start event is recorded before its batch's searches, its done
// event after its record; a gathered frame is not finished until then.
struct BatchExec : HipExec {
  struct Item {
    Resident* r;
    int64_t req;
    hipEvent_t start, done;
  };
  int max_batch = 2;
  std::vector<vy_batch_ctx*> bctx;        // one per stream
  std::vector<std::vector<Item>> gather;  // per stream
  std::vector<int> gather_filter;
  std::vector<uint32_t> gather_tiles;
  std::vector<int> open;                  // per stream: frames enqueued and not seen finished
  std::vector<int> stream_of;             // per request: its stream
  std::vector<char> enqueued;             // per request: its batch has been enqueued
  std::vector<vy_view> views;

  static uint32_t tiles_of(const vy_session& ss) {
    return (uint32_t)(((ss.width + 15) / 16) * ((ss.height + 15) / 16));
  }

  // a session's next frame may join the stream's batch only if it has none there
  bool can_take(const Resident& r, int k) const {
    for (const Item& it : gather[k])
      if (it.r == &r) return false;
    return true;
  }

  int dispatch(Resident& r, int64_t i, int k, Ticket* t, int32_t* status) {
    const vy_session& ss = sessions[r.session];
    const SessionPlan& p = plans[r.session];
    hipStream_t st = streams[k];
    if (!r.cut && cut_create_on(ss.scene, (char*)r.mem, p.cut_bytes, st, false, &r.cut) != VY_OK) return VY_ERR_HIP;
    if (pool->size() < 2) return fail(VY_ERR_HIP, "vy_server_run: event pool exhausted");
    // a full batch, or one of the other filter, or too many tiles: enqueue it first
    if (!gather[k].empty() && ((int)gather[k].size() >= max_batch || gather_filter[k] != ss.alpha_filter ||
                               gather_tiles[k] + tiles_of(ss) > VY_BATCH_MAX_TILES))
      if (int rc = flush_stream(k)) return rc;
    t->start = pool->back();
    pool->pop_back();
    t->done = pool->back();
    pool->pop_back();
    gather[k].push_back(Item{&r, i, t->start, t->done});
    gather_filter[k] = ss.alpha_filter;
    gather_tiles[k] += tiles_of(ss);
    stream_of[i] = k;
    enqueued[i] = 0;
    *status = VY_OK;
    return VY_OK;
  }

  int poll(const Ticket& t, Outcome* o) {
    if (!enqueued[t.req]) return 0;   // still gathering: its events are not recorded yet
    const int rc = HipExec::poll(t, o);
    if (rc == 1) --open[stream_of[t.req]];
    return rc;
  }

  int flush_stream(int k) {
    std::vector<Item>& g = gather[k];
    if (g.empty()) return VY_OK;
    hipStream_t st = streams[k];
    views.clear();
    int err = VY_OK;
    for (const Item& it : g) VY_HIP(hipEventRecord(it.start, st));
    // a record may hold an earlier attempt of its frame: the hash is summed into it
    for (const Item& it : g) VY_HIP(hipMemsetAsync(stats + it.req, 0, sizeof(vy_frame_stats), st));
    for (const Item& it : g) {
      Resident& r = *it.r;
      const vy_frame_req& q = reqs[it.req];
      const vy_session& ss = sessions[r.session];
      const int rc = vy_lod_cut(ss.scene, &q.cam, ss.tau, r.has_cut ? r.cut : nullptr, r.cut, VY_CUT_FRONTIER, st);
      if (rc == VY_ERR_HIP) return rc;
      if (rc != VY_OK) err = rc;
      r.has_cut = true;
      const SessionPlan& p = plans[r.session];
      views.push_back(vy_view{ss.scene, r.cut, q.cam, q.image ? q.image : (float*)((char*)r.mem + p.cut_bytes)});
    }
    if (err == VY_OK) {
      vy_render_opts o;
      memset(&o, 0, sizeof(o));
      o.alpha_filter = gather_filter[k];
      err = vy_render_batch(views.data(), (int32_t)views.size(), &o, bctx[k], st);
      if (err == VY_ERR_HIP) return err;
    }
    for (size_t j = 0; j < g.size(); ++j) {
      const Item& it = g[j];
      const vy_session& ss = sessions[it.r->session];
      if (err == VY_OK) {
        const int rc = batch_frame_finish(it.r->cut, bctx[k], views[j].image, ss.width, ss.height, stats + it.req, st);
        if (rc != VY_OK) return rc;
      }
      VY_HIP(hipMemcpyAsync(host_stats + it.req, stats + it.req, sizeof(vy_frame_stats), hipMemcpyDeviceToHost, st));
      VY_HIP(hipEventRecord(it.done, st));
    }
    if (err != VY_OK) return err;
    for (const Item& it : g) enqueued[it.req] = 1;
    open[k] += (int)g.size();
    g.clear();
    gather_tiles[k] = 0;
    return VY_OK;
  }

  int flush() {
    for (int k = 0; k < n_streams; ++k)
      if (!gather[k].empty() && ((int)gather[k].size() >= max_batch || open[k] == 0))
        if (int rc = flush_stream(k)) return rc;
    return VY_OK;
  }

  void drop_render(Resident&) {}
  void release(Resident& r) {
    if (r.cut) vy_cut_free(r.cut);
    r.cut = nullptr;
  }
};

// Model: a frame keeps its stream busy for its service time; a session's
// render block is 16 bytes per pair of capacity, and a frame overflows when
// it needs more pairs than the capacity it was dispatched with.
struct SimExec {
  const double* service;
  const uint32_t* need_pairs;             // optional: a frame overflows a pair capacity below this
  std::vector<double> stream_free;
  std::multiset<double> done_times;
  std::vector<int64_t> cap_of;            // per request: pair capacity it was dispatched with
  double clock = 0;

  double now() const { return clock; }
  size_t render_bytes(int, int64_t, int64_t q) const { return (size_t)q * 16; }

  int dispatch(Resident& r, int64_t i, int k, Ticket* t, int32_t* status) {
    t->t_start = std::max(clock, stream_free[k]);
    t->t_done = t->t_start + service[i];
    stream_free[k] = t->t_done;
    done_times.insert(t->t_done);
    cap_of[i] = r.cap_pairs;
    *status = VY_OK;
    return VY_OK;
  }

  int poll(const Ticket& t, Outcome* o) {
    if (t.t_done > clock) return 0;
    o->t_start = t.t_start;
    o->t_done = t.t_done;
    if (need_pairs && (int64_t)need_pairs[t.req] > cap_of[t.req]) {
      o->flags = kFlagPairs;
      o->n_pairs = need_pairs[t.req];
    }
    done_times.erase(done_times.find(t.t_done));
    return 1;
  }

  void recycle(Ticket&) {}
  void drop_render(Resident&) {}
  void release(Resident&) {}
  void drain() {}
  bool can_take(const Resident&, int) const { return true; }
  int flush() { return VY_OK; }

  int wait(double next_arrival, int64_t) {
    const double next_done = done_times.empty() ? INFINITY : *done_times.begin();
    const double t = std::min(next_arrival, next_done);
    if (!std::isfinite(t)) return fail(VY_ERR_STATE, "vy_server_simulate: no event to wait for");
    clock = std::max(clock, t);
    return VY_OK;
  }
};

// ---------------------------------------------------------------- server ----

struct Server {
  uint32_t magic = kServerMagic;
  Arena* arena = nullptr;
  std::vector<hipStream_t> streams;
  int max_inflight = 1, max_viewers = 1;
  int max_batch = 0;
  int64_t batch_g = 0, batch_pairs = 0;
  std::vector<hipEvent_t> pool;
  hipEvent_t t0_event = nullptr;
  RunCounters last;
};

int check_config(const vy_server_config* c, bool need_streams, const char* who) {
  if (!c || !as_arena(c->arena)) return fail(VY_ERR_ARG, "%s: NULL config or arena", who);
  if (c->n_streams < 1 || c->n_streams > 16) return fail(VY_ERR_ARG, "%s: n_streams must be 1..16", who);
  if (c->max_inflight < 1 || c->max_inflight > 64) return fail(VY_ERR_ARG, "%s: max_inflight must be 1..64", who);
  if (c->max_viewers < 1 || c->max_viewers > 4096) return fail(VY_ERR_ARG, "%s: max_viewers must be 1..4096", who);
  if (c->max_batch < 0 || c->max_batch > VY_BATCH_MAX_VIEWS || c->reserved != 0)
    return fail(VY_ERR_ARG, "%s: max_batch must be 0..%d (reserved 0)", who, VY_BATCH_MAX_VIEWS);
  if (c->max_batch > 1 && (c->batch_gaussians < 1 || c->batch_gaussians > 0x7FFFFFFF || c->batch_pairs < 1 ||
                           c->batch_pairs > 0x7FFFFFFF))
    return fail(VY_ERR_ARG, "%s: batching needs batch_gaussians and batch_pairs in 1..2^31-1", who);
  if (need_streams) {
    if (!c->streams) return fail(VY_ERR_ARG, "%s: NULL streams", who);
    for (int i = 0; i < c->n_streams; ++i) {
      if (!c->streams[i]) return fail(VY_ERR_ARG, "%s: stream %d is NULL (the null stream is not allowed)", who, i);
      for (int j = 0; j < i; ++j)
        if (c->streams[j] == c->streams[i]) return fail(VY_ERR_ARG, "%s: streams %d and %d are the same", who, j, i);
    }
  }
  return VY_OK;
}

// Requests: session index in range, arrivals finite, >= 0 and non-decreasing.
int check_trace(int32_t n_sessions, const vy_frame_req* reqs, int64_t n_reqs, const vy_frame_result* results,
                const char* who) {
  if (n_reqs < 0 || n_sessions < 0 || (n_reqs > 0 && (!reqs || !results || n_sessions < 1)))
    return fail(VY_ERR_ARG, "%s: bad trace arguments", who);
  double last = 0;
  for (int64_t i = 0; i < n_reqs; ++i) {
    const vy_frame_req& q = reqs[i];
    if (q.session < 0 || q.session >= n_sessions) return fail(VY_ERR_ARG, "%s: request %lld: bad session", who, (long long)i);
    if (!std::isfinite(q.t_arrival) || q.t_arrival < last)
      return fail(VY_ERR_ARG, "%s: request %lld: arrival times must be finite, >= 0 and non-decreasing", who,
                  (long long)i);
    last = q.t_arrival;
  }
  return VY_OK;
}

}  // namespace

extern "C" {

int vy_arena_create(void* base, size_t bytes, vy_arena** out) {
  if (!out) return fail(VY_ERR_ARG, "vy_arena_create: NULL out");
  *out = nullptr;
  if (!base || ((uintptr_t)base % kGranule) != 0 || bytes < kGranule)
    return fail(VY_ERR_ARG, "vy_arena_create: base must be non-NULL and 256-byte aligned, bytes >= 256");
  Arena* a = new (std::nothrow) Arena();
  if (!a) return fail(VY_ERR_ARG, "vy_arena_create: out of host memory");
  a->base = (uintptr_t)base;
  a->bytes = bytes / kGranule * kGranule;
  a->free_blocks.emplace(0, a->bytes);
  *out = (vy_arena*)a;
  return VY_OK;
}

int vy_arena_free(vy_arena* arena) {
  if (!arena) return VY_OK;
  Arena* a = as_arena(arena);
  if (!a) return fail(VY_ERR_ARG, "vy_arena_free: not an arena");
  a->magic = 0;
  delete a;
  return VY_OK;
}

int vy_arena_alloc(vy_arena* arena, size_t bytes, void** out) {
  Arena* a = as_arena(arena);
  if (!a || !out) return fail(VY_ERR_ARG, "vy_arena_alloc: bad argument");
  return a->alloc(bytes, out);
}

int vy_arena_release(vy_arena* arena, void* ptr) {
  Arena* a = as_arena(arena);
  if (!a) return fail(VY_ERR_ARG, "vy_arena_release: bad argument");
  return a->release(ptr);
}

int vy_arena_stats(const vy_arena* arena, size_t* used, size_t* largest_free, int64_t* n_live, int64_t* n_free_blocks) {
  const Arena* a = as_arena(arena);
  if (!a) return fail(VY_ERR_ARG, "vy_arena_stats: bad argument");
  if (used) *used = a->used;
  if (largest_free) *largest_free = a->largest();
  if (n_live) *n_live = (int64_t)a->live.size();
  if (n_free_blocks) *n_free_blocks = (int64_t)a->free_blocks.size();
  return VY_OK;
}

size_t vy_session_bytes(const vy_session* session) {
  SessionPlan p;
  return plan_session(session, &p) ? p.total : 0;
}

int vy_server_create(const vy_server_config* config, vy_server** out) {
  if (!out) return fail(VY_ERR_ARG, "vy_server_create: NULL out");
  *out = nullptr;
  if (int rc = check_config(config, true, "vy_server_create")) return rc;
  Server* s = new (std::nothrow) Server();
  if (!s) return fail(VY_ERR_ARG, "vy_server_create: out of host memory");
  s->arena = as_arena(config->arena);
  for (int i = 0; i < config->n_streams; ++i) s->streams.push_back((hipStream_t)config->streams[i]);
  s->max_inflight = config->max_inflight;
  s->max_viewers = config->max_viewers;
  s->max_batch = config->max_batch > 1 ? config->max_batch : 0;
  s->batch_g = config->batch_gaussians;
  s->batch_pairs = config->batch_pairs;
  const int n_ev = 2 * config->n_streams * config->max_inflight;
  hipError_t e = hipEventCreate(&s->t0_event);
  for (int i = 0; i < n_ev && e == hipSuccess; ++i) {
    hipEvent_t ev;
    e = hipEventCreate(&ev);
    if (e == hipSuccess) s->pool.push_back(ev);
  }
  if (e != hipSuccess) {
    vy_server_free((vy_server*)s);
    return fail(VY_ERR_HIP, "vy_server_create: hipEventCreate: %s", hipGetErrorString(e));
  }
  *out = (vy_server*)s;
  return VY_OK;
}

int vy_server_free(vy_server* server) {
  Server* s = (Server*)server;
  if (!s) return VY_OK;
  if (s->magic != kServerMagic) return fail(VY_ERR_ARG, "vy_server_free: not a server");
  for (hipEvent_t e : s->pool) (void)hipEventDestroy(e);
  if (s->t0_event) (void)hipEventDestroy(s->t0_event);
  s->magic = 0;
  delete s;
  return VY_OK;
}

int vy_server_run(vy_server* server, const vy_session* sessions, int32_t n_sessions, const vy_frame_req* reqs,
                  int64_t n_reqs, int32_t flags, vy_frame_stats* stats, vy_frame_result* results) {
  Server* s = (Server*)server;
  if (!s || s->magic != kServerMagic) return fail(VY_ERR_ARG, "vy_server_run: bad server");
  if (int rc = check_trace(n_sessions, reqs, n_reqs, results, "vy_server_run")) return rc;
  if (n_sessions > 0 && !sessions) return fail(VY_ERR_ARG, "vy_server_run: NULL sessions");
  const bool batched = s->max_batch > 1;
  std::vector<SessionPlan> plans(n_sessions);
  for (int i = 0; i < n_sessions; ++i)
    if (!plan_session(&sessions[i], &plans[i], batched))
      return fail(VY_ERR_ARG, "vy_server_run: session %d is invalid", i);
  const size_t rec_bytes = round_up(sizeof(vy_frame_stats) * (size_t)std::max<int64_t>(n_reqs, 1), kGranule);
  const size_t batch_bytes =
      batched ? round_up(vy_batch_workspace_bytes(s->max_batch, s->batch_g, VY_BATCH_MAX_TILES, s->batch_pairs),
                         kGranule)
              : 0;
  const size_t reserve = (stats ? 0 : rec_bytes) + batch_bytes * s->streams.size();
  if (reserve > s->arena->bytes)
    return fail(VY_ERR_CAPACITY, "vy_server_run: the batch contexts and records need %zu bytes, the arena has %zu",
                reserve, s->arena->bytes);
  const size_t room = s->arena->bytes - reserve;
  for (int64_t i = 0; i < n_reqs; ++i) {
    const vy_session& ss = sessions[reqs[i].session];
    if (reqs[i].cam.width != ss.width || reqs[i].cam.height != ss.height || reqs[i].reserved != 0)
      return fail(VY_ERR_ARG, "vy_server_run: request %lld: camera size differs from its session's", (long long)i);
    if (plans[reqs[i].session].total > room || rec_bytes > s->arena->bytes)
      return fail(VY_ERR_CAPACITY, "vy_server_run: session %d needs %zu bytes, the arena has room for %zu",
                  reqs[i].session, plans[reqs[i].session].total, room);
  }
  if (!s->arena->live.empty()) return fail(VY_ERR_STATE, "vy_server_run: the arena has live blocks");
  for (int64_t i = 0; i < n_reqs; ++i) {
    results[i] = vy_frame_result();
    results[i].stream = -1;
  }
  s->last = RunCounters();
  if (n_reqs == 0) return VY_OK;
  const int ns = (int)s->streams.size();
  // frame records: the caller's, or a block of the arena; pinned host copies
  void* own = nullptr;
  if (!stats) {
    if (int rc = s->arena->alloc(rec_bytes, &own)) return rc;
    stats = (vy_frame_stats*)own;
  }
  vy_frame_stats* host = nullptr;
  hipError_t e = hipHostMalloc((void**)&host, sizeof(vy_frame_stats) * n_reqs, hipHostMallocDefault);
  if (e != hipSuccess) {
    if (own) (void)s->arena->release(own);
    return fail(VY_ERR_HIP, "vy_server_run: hipHostMalloc: %s", hipGetErrorString(e));
  }
  BatchExec ex;
  ex.sessions = sessions;
  ex.plans = plans.data();
  ex.reqs = reqs;
  ex.stats = stats;
  ex.host_stats = host;
  ex.streams = s->streams.data();
  ex.n_streams = ns;
  ex.pool = &s->pool;
  ex.t0_event = s->t0_event;
  int rc = VY_OK;
  // batching: one batch context per stream, carved from the arena for the run
  std::vector<void*> bmem;
  if (batched) {
    ex.max_batch = s->max_batch;
    ex.gather.assign(ns, {});
    ex.gather_filter.assign(ns, 0);
    ex.gather_tiles.assign(ns, 0);
    ex.open.assign(ns, 0);
    ex.stream_of.assign(n_reqs, 0);
    ex.enqueued.assign(n_reqs, 0);
    for (int k = 0; k < ns && rc == VY_OK; ++k) {
      void* m = nullptr;
      vy_batch_ctx* b = nullptr;
      rc = s->arena->alloc(batch_bytes, &m);
      if (rc == VY_OK) {
        bmem.push_back(m);
        rc = vy_batch_ctx_create(s->max_batch, s->batch_g, VY_BATCH_MAX_TILES, s->batch_pairs, m, batch_bytes, &b);
      }
      if (rc == VY_OK) ex.bctx.push_back(b);
    }
  }
  if (rc == VY_OK) e = hipMemsetAsync(stats, 0, sizeof(vy_frame_stats) * n_reqs, s->streams[0]);
  for (int k = 0; k < ns && e == hipSuccess; ++k) e = hipStreamSynchronize(s->streams[k]);
  if (e == hipSuccess) e = hipEventRecord(s->t0_event, s->streams[0]);
  if (e == hipSuccess) e = hipEventSynchronize(s->t0_event);
  if (rc != VY_OK) {
    // a batch context could not be set up: nothing ran
  } else if (e != hipSuccess) {
    rc = fail(VY_ERR_HIP, "vy_server_run: start: %s", hipGetErrorString(e));
  } else if (batched) {
    ex.t0 = host_seconds();
    Runner<BatchExec> run(ex, s->arena, ns, s->max_inflight, s->max_viewers, reqs, n_reqs, n_sessions, plans.data(),
                          (flags & VY_RUN_REALTIME) != 0, results);
    rc = run.run();
    s->last = run.cnt;
  } else {
    HipExec& hx = ex;
    hx.t0 = host_seconds();
    Runner<HipExec> run(hx, s->arena, ns, s->max_inflight, s->max_viewers, reqs, n_reqs, n_sessions, plans.data(),
                        (flags & VY_RUN_REALTIME) != 0, results);
    rc = run.run();
    s->last = run.cnt;
  }
  ex.drain();
  for (vy_batch_ctx* b : ex.bctx) (void)vy_batch_ctx_free(b);
  for (void* m : bmem) (void)s->arena->release(m);
  (void)hipHostFree(host);
  if (own) (void)s->arena->release(own);
  return rc;
}

int vy_server_last_run(const vy_server* server, int64_t* n_admitted, int64_t* n_waited, int64_t* peak_resident,
                       size_t* peak_bytes, int64_t* n_regrown, int64_t* n_redone) {
  const Server* s = (const Server*)server;
  if (!s || s->magic != kServerMagic) return fail(VY_ERR_ARG, "vy_server_last_run: bad server");
  if (n_admitted) *n_admitted = s->last.admitted;
  if (n_waited) *n_waited = s->last.waited;
  if (peak_resident) *peak_resident = s->last.peak_resident;
  if (peak_bytes) *peak_bytes = s->last.peak_bytes;
  if (n_regrown) *n_regrown = s->last.regrown;
  if (n_redone) *n_redone = s->last.redone;
  return VY_OK;
}

int vy_server_simulate(const vy_server_config* config, const int64_t* session_bytes, const int64_t* pair_capacity,
                       int32_t n_sessions, const vy_frame_req* reqs, int64_t n_reqs, const double* service_s,
                       const uint32_t* need_pairs, int32_t flags, vy_frame_result* results, int64_t* counters) {
  if (int rc = check_config(config, false, "vy_server_simulate")) return rc;
  if (int rc = check_trace(n_sessions, reqs, n_reqs, results, "vy_server_simulate")) return rc;
  if (n_reqs > 0 && (!session_bytes || !service_s)) return fail(VY_ERR_ARG, "vy_server_simulate: NULL arrays");
  if (need_pairs && !pair_capacity)
    return fail(VY_ERR_ARG, "vy_server_simulate: need_pairs requires pair capacities");
  Arena* arena = as_arena(config->arena);
  std::vector<SessionPlan> plans(n_sessions);
  for (int i = 0; i < n_sessions; ++i) {
    SessionPlan& p = plans[i];
    if (session_bytes[i] < 1 || (pair_capacity && (pair_capacity[i] < 1 || pair_capacity[i] > kMaxPairsCap)))
      return fail(VY_ERR_ARG, "vy_server_simulate: session %d: bytes and pair capacity must be > 0", i);
    p.fixed = (size_t)session_bytes[i];
    p.max_pairs = pair_capacity ? pair_capacity[i] : 0;
    p.grow_pairs = need_pairs != nullptr;
    p.render_bytes = (size_t)p.max_pairs * 16;
    p.total = p.fixed + p.render_bytes;
  }
  for (int64_t i = 0; i < n_reqs; ++i) {
    if (!(service_s[i] >= 0) || !std::isfinite(service_s[i]))
      return fail(VY_ERR_ARG, "vy_server_simulate: request %lld: service time must be finite and >= 0", (long long)i);
    if (plans[reqs[i].session].total > arena->bytes)
      return fail(VY_ERR_CAPACITY, "vy_server_simulate: session %d does not fit the arena", reqs[i].session);
  }
  if (!arena->live.empty()) return fail(VY_ERR_STATE, "vy_server_simulate: the arena has live blocks");
  for (int64_t i = 0; i < n_reqs; ++i) {
    results[i] = vy_frame_result();
    results[i].stream = -1;
  }
  SimExec ex;
  ex.service = service_s;
  ex.need_pairs = need_pairs;
  ex.cap_of.assign(n_reqs, 0);
  ex.stream_free.assign(config->n_streams, 0.0);
  Runner<SimExec> run(ex, arena, config->n_streams, config->max_inflight, config->max_viewers, reqs, n_reqs,
                      n_sessions, plans.data(), (flags & VY_RUN_REALTIME) != 0, results);
  const int rc = run.run();
  if (counters) {
    counters[0] = run.cnt.admitted;
    counters[1] = run.cnt.waited;
    counters[2] = run.cnt.peak_resident;
    counters[3] = (int64_t)run.cnt.peak_bytes;
    counters[4] = run.cnt.regrown;
    counters[5] = run.cnt.redone;
  }
  return rc;
}

}  // extern "C"
