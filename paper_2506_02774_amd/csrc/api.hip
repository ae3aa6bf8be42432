// Error reporting, version and launch timing for the Voyager HIP library.
#include <cstdarg>
#include <cstring>
#include <vector>

#include "vy_common.hpp"

namespace vy {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

uint32_t next_epoch(uint32_t& epoch) {
  epoch = (epoch + 1) & 0xFFFFFFu;
  if (epoch == 0) epoch = 1;
  return epoch;
}

// ---------------------------------------------------------------- timing ----

struct ProfRec {
  int stage;
  hipEvent_t a, b;
};

static thread_local bool g_prof_on = false;
static thread_local std::vector<ProfRec>* g_prof = nullptr;
static thread_local int64_t g_prof_cap = 0;
static thread_local hipEvent_t g_pending_start = nullptr;

void prof_mark(int stage, hipStream_t s, bool end) {
  if (!g_prof_on || !g_prof) return;
  if (!end) {
    if ((int64_t)g_prof->size() >= g_prof_cap) { g_pending_start = nullptr; return; }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) { g_pending_start = nullptr; return; }
    hipEventRecord(e, s);
    g_pending_start = e;
  } else {
    if (!g_pending_start) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) { hipEventDestroy(g_pending_start); g_pending_start = nullptr; return; }
    hipEventRecord(e, s);
    g_prof->push_back({stage, g_pending_start, e});
    g_pending_start = nullptr;
  }
}

}  // namespace vy

using namespace vy;

extern "C" {

const char* vy_last_error(void) { return vy::g_err; }
const char* vy_version(void) { return "voyager-mi355x 0.1 (gfx950)"; }

static const char* kStageNames[VY_NUM_STAGES] = {
    "lod_setup", "lod_flat", "lod_classify", "lod_traverse", "lod_compact", "render_setup", "project",
    "depth_sort", "pair_scan", "emit", "tile_sort", "ranges", "blend"};

const char* vy_stage_name(int stage) {
  if (stage < 0 || stage >= VY_NUM_STAGES) return "?";
  return kStageNames[stage];
}

int vy_profile_begin(int64_t capacity) {
  if (capacity <= 0) return fail(VY_ERR_ARG, "vy_profile_begin: capacity must be > 0");
  if (!g_prof) g_prof = new std::vector<ProfRec>();
  for (auto& r : *g_prof) { hipEventDestroy(r.a); hipEventDestroy(r.b); }
  g_prof->clear();
  g_prof->reserve((size_t)capacity);
  g_prof_cap = capacity;
  g_prof_on = true;
  return VY_OK;
}

int vy_profile_end(double* stage_ms, int64_t* stage_launches) {
  g_prof_on = false;
  if (!g_prof) return fail(VY_ERR_STATE, "vy_profile_end without vy_profile_begin");
  for (int i = 0; i < VY_NUM_STAGES; ++i) {
    if (stage_ms) stage_ms[i] = 0;
    if (stage_launches) stage_launches[i] = 0;
  }
  int rc = VY_OK;
  for (auto& r : *g_prof) {
    if (hipEventSynchronize(r.b) != hipSuccess) rc = fail(VY_ERR_HIP, "hipEventSynchronize failed");
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) ms = 0;
    if (stage_ms) stage_ms[r.stage] += ms;
    if (stage_launches) stage_launches[r.stage] += 1;
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  g_prof->clear();
  return rc;
}

}  // extern "C"
