// Internal helpers shared by the HIP translation units of librad.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/rad.h"

namespace rad {

// Thread-local message of the last failing call (returned by rad_last_error).
void set_error(const std::string& msg);
void clear_error();

#define RAD_HIP_CHECK(expr)                                                      \
  do {                                                                           \
    hipError_t _e = (expr);                                                      \
    if (_e != hipSuccess) {                                                      \
      ::rad::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));       \
      return RAD_EHIP;                                                           \
    }                                                                            \
  } while (0)

#define RAD_REQUIRE(cond, code, msg)                                             \
  do {                                                                           \
    if (!(cond)) {                                                               \
      ::rad::set_error(msg);                                                     \
      return (code);                                                             \
    }                                                                            \
  } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Simple bump allocator over a caller-provided workspace.
struct Carve {
  char* base;
  size_t size;
  size_t used = 0;
  bool ok = true;
  Carve(void* p, size_t n) : base(static_cast<char*>(p)), size(n) {}
  template <class T>
  T* take(size_t count) {
    size_t off = align_up(used, 256);
    size_t bytes = align_up(count * sizeof(T), 256);
    if (base == nullptr || off + bytes > size) {
      ok = false;
      used = off + bytes;
      return nullptr;
    }
    used = off + bytes;
    return reinterpret_cast<T*>(base + off);
  }
};

// One C-ABI call as a named roctx range, so that a marker trace
// (rocprofv3 --marker-trace) shows each call around the kernels it enqueued.
// Without an attached tool the push and pop return at once.
struct ApiRange {
  explicit ApiRange(const char* name) { roctxRangePushA(name); }
  ~ApiRange() { roctxRangePop(); }
  ApiRange(const ApiRange&) = delete;
  ApiRange& operator=(const ApiRange&) = delete;
};

// Per-launch kernel timing (see profile.hip).
bool prof_enabled(int kind);
hipEvent_t prof_event();
void prof_push(int kind, hipEvent_t a, hipEvent_t b, double flops, double bytes);

// Brackets one launch with events when profiling is on.
struct ProfScope {
  hipStream_t s;
  int kind;
  double flops, bytes;
  hipEvent_t a = nullptr;
  ProfScope(hipStream_t st, int k, double f, double b) : s(st), kind(k), flops(f), bytes(b) {
    if (prof_enabled(k)) {
      a = prof_event();
      if (a) hipEventRecord(a, s);
    }
  }
  ~ProfScope() {
    if (a) {
      hipEvent_t b = prof_event();
      if (b) hipEventRecord(b, s);
      prof_push(kind, a, b, flops, bytes);
    }
  }
};

// Second stream of the calling host thread on the current device (created on
// first use, default priority, never destroyed).  `dst` waits for everything
// enqueued on `src` so far via event ev[k]; an event is re-recorded only
// after the wait on its previous record has been enqueued.
struct SideStream {
  hipStream_t s2;
  hipEvent_t ev[6];
};
hipError_t side_stream(SideStream** out);
bool lookahead_enabled();  // tuning: split trailing updates over the two streams
inline hipError_t stream_wait(hipStream_t dst, hipStream_t src, hipEvent_t ev) {
  hipError_t e = hipEventRecord(ev, src);
  if (e != hipSuccess) return e;
  return hipStreamWaitEvent(dst, ev, 0);
}

// Device status codes raised by kernels (stored in an int32 flag; the
// smallest (most negative) code wins via atomicMin).
__device__ inline void raise_status(int* flag, int code) { atomicMin(flag, code); }

// The hardware hands workgroup k of a launch to XCD k % 8, and each XCD has
// its own L2: this maps dispatch index pid to a logical index such that each
// XCD owns a contiguous range of the total.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int xcd_contiguous(int pid, int total) {
  const int q = total / NUM_XCD, rem = total % NUM_XCD;
  const int x = pid % NUM_XCD, loc = pid / NUM_XCD;
  return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + loc;
}

// tile pair (I, J), I <= J, of index p in the row-wise enumeration of the
// upper triangle of a t x t tile grid
__device__ inline void pair_from_index(long p, int t, int& I, int& J) {
  // row-wise enumeration of the upper triangle (I <= J) of a t x t tile grid
  double tt = 2.0 * t + 1.0;
  int i = static_cast<int>((tt - sqrt(tt * tt - 8.0 * static_cast<double>(p))) * 0.5);
  if (i < 0) i = 0;
  if (i > t - 1) i = t - 1;
  auto start = [t](long r) { return r * t - r * (r - 1) / 2; };
  while (i > 0 && start(i) > p) --i;
  while (i + 1 < t && start(i + 1) <= p) ++i;
  I = i;
  J = static_cast<int>(i + (p - start(i)));
}


// Non-negative doubles order like their bit patterns: atomicMax on the
// bits gives an order-independent, reproducible max.
__device__ inline void atomic_max_nonneg(double* p, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(p),
            static_cast<unsigned long long>(__double_as_longlong(v)));
}

}  // namespace rad
