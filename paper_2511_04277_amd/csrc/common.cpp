// Error strings and thread-local error state of the C ABI.
#include <string>

#include "../../include/rad.h"

namespace rad {
namespace {
thread_local std::string g_last_error;
}
void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }
}  // namespace rad

extern "C" const char* rad_last_error(void) { return rad::g_last_error.c_str(); }

extern "C" int32_t rad_version(void) { return 100; }

extern "C" const char* rad_status_string(int32_t code) {
  switch (code) {
    case RAD_OK: return "ok";
    case RAD_WNOTCONVERGED: return "tolerance not met within the iteration limit";
    case RAD_EINVAL: return "invalid argument";
    case RAD_ENONFINITE: return "non-finite or out-of-range input value";
    case RAD_EZEROROW: return "a view-factor row sums to zero";
    case RAD_ESINGULAR: return "singular pivot block";
    case RAD_EHIP: return "HIP runtime error";
    case RAD_EWORKSPACE: return "workspace too small or misaligned";
    default: return "unknown status";
  }
}
