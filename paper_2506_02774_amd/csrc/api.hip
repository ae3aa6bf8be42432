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
  int slot;
};

// Events are created once by vy_profile_begin (2 per launch slot), so that a
// recorded launch costs two hipEventRecord calls and nothing else.
static thread_local bool g_prof_on = false;
static thread_local std::vector<ProfRec>* g_prof = nullptr;
static thread_local std::vector<hipEvent_t>* g_events = nullptr;
static thread_local int64_t g_prof_cap = 0;
static thread_local int g_open_slot = -1;

void prof_mark(int stage, hipStream_t s, bool end) {
  if (!g_prof_on || !g_prof || !g_events) return;
  if (!end) {
    g_open_slot = -1;
    if ((int64_t)g_prof->size() >= g_prof_cap) return;
    const int slot = (int)g_prof->size();
    if (hipEventRecord((*g_events)[2 * slot], s) != hipSuccess) return;
    g_open_slot = slot;
  } else {
    if (g_open_slot < 0) return;
    if (hipEventRecord((*g_events)[2 * g_open_slot + 1], s) == hipSuccess) g_prof->push_back({stage, g_open_slot});
    g_open_slot = -1;
  }
}

static void prof_release() {
  if (g_events) {
    for (hipEvent_t e : *g_events) (void)hipEventDestroy(e);
    g_events->clear();
  }
  if (g_prof) g_prof->clear();
  g_prof_cap = 0;
}

}  // namespace vy

using namespace vy;

extern "C" {

const char* vy_last_error(void) { return vy::g_err; }
const char* vy_version(void) { return "voyager-mi355x 0.1 (gfx950)"; }

static const char* kStageNames[VY_NUM_STAGES] = {
    "lod_setup", "lod_flat", "lod_classify", "lod_traverse", "lod_compact", "render_setup", "project",
    "depth_sort", "pair_scan", "emit", "tile_sort", "ranges", "blend_plan", "blend", "bwd_blend", "bwd_project"};

const char* vy_stage_name(int stage) {
  if (stage < 0 || stage >= VY_NUM_STAGES) return "?";
  return kStageNames[stage];
}

int vy_profile_begin(int64_t capacity) {
  if (capacity <= 0 || capacity > (1 << 22)) return fail(VY_ERR_ARG, "vy_profile_begin: capacity out of range");
  if (!g_prof) g_prof = new std::vector<ProfRec>();
  if (!g_events) g_events = new std::vector<hipEvent_t>();
  prof_release();
  g_prof->reserve((size_t)capacity);
  g_events->reserve(2 * (size_t)capacity);
  for (int64_t i = 0; i < 2 * capacity; ++i) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
      prof_release();
      return fail(VY_ERR_HIP, "vy_profile_begin: hipEventCreate failed");
    }
    g_events->push_back(e);
  }
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
    hipEvent_t a = (*g_events)[2 * r.slot], b = (*g_events)[2 * r.slot + 1];
    if (hipEventSynchronize(b) != hipSuccess) rc = fail(VY_ERR_HIP, "hipEventSynchronize failed");
    float ms = 0;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) ms = 0;
    if (stage_ms) stage_ms[r.stage] += ms;
    if (stage_launches) stage_launches[r.stage] += 1;
  }
  prof_release();
  return rc;
}

}  // extern "C"
