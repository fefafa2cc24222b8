// Optional per-launch timing of the hot kernels with HIP events.
//
// When enabled (rad_profile_enable, per host thread), every launch of a
// profiled kernel of a selected kind (rad_profile_kinds) is bracketed by two
// events on its stream; rad_profile_read
// waits for them and reports launches, summed device time and the launches'
// algorithmic flops / bytes per kernel kind.
#include <vector>

#include "common.h"

namespace rad {
namespace {
struct Rec {
  hipEvent_t a, b;
  int kind;
  double flops, bytes;
};
thread_local bool g_on = false;
thread_local uint32_t g_mask = 0xffffffffu;
thread_local std::vector<Rec> g_recs;
thread_local std::vector<hipEvent_t> g_pool;
}  // namespace

bool prof_enabled(int kind) { return g_on && kind >= 0 && kind < 32 && ((g_mask >> kind) & 1u); }

hipEvent_t prof_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void prof_push(int kind, hipEvent_t a, hipEvent_t b, double flops, double bytes) {
  if (a && b) g_recs.push_back(Rec{a, b, kind, flops, bytes});
}

}  // namespace rad

using namespace rad;

extern "C" int32_t rad_profile_enable(int32_t on) {
  g_on = on != 0;
  return RAD_OK;
}

extern "C" int32_t rad_profile_kinds(uint32_t mask) {
  g_mask = mask;
  return RAD_OK;
}

extern "C" int32_t rad_profile_read(rad_kernel_profile* out, int32_t count) {
  clear_error();
  RAD_REQUIRE(out && count >= 0, RAD_EINVAL, "rad_profile_read: NULL output");
  for (int k = 0; k < count; ++k) out[k] = rad_kernel_profile{0, 0.0, 0.0, 0.0};
  int32_t rc = RAD_OK;
  for (const Rec& r : g_recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      set_error("rad_profile_read: event query failed");
      rc = RAD_EHIP;
    } else if (r.kind >= 0 && r.kind < count) {
      out[r.kind].launches += 1;
      out[r.kind].total_ms += ms;
      out[r.kind].flops += r.flops;
      out[r.kind].bytes += r.bytes;
    }
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  return rc;
}
