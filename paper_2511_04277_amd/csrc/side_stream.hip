// A second stream per device and host thread, for work that overlaps the
// caller's stream inside one call (fork and join through events).
#include <unordered_map>

#include "common.h"

namespace rad {
namespace {
thread_local std::unordered_map<int, SideStream> g_side;
}

hipError_t side_stream(SideStream** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  auto it = g_side.find(dev);
  if (it == g_side.end()) {
    SideStream ss{};
    // default priority; no implicit ordering with the null stream (events order it)
    e = hipStreamCreateWithFlags(&ss.s2, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    for (hipEvent_t& ev : ss.ev) {
      e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
    it = g_side.emplace(dev, ss).first;
  }
  *out = &it->second;
  return hipSuccess;
}

}  // namespace rad
