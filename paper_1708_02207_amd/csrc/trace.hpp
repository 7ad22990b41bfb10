// roctx ranges around the host-side phases of the library (builds and their
// levels, full and partial Root to Leaves, refinement sweeps, further loads,
// served batches), so that a trace with markers shows which phase issued
// which kernels.  A range is pushed on the calling thread and popped when
// the object goes out of scope.  Without a profiler attached roctx calls
// return at once.  Under stream capture the ranges mark the capture, not the
// replays.
#pragma once
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdio>

namespace hdd {

class Range {
 public:
  explicit Range(const char* name) { roctxRangePushA(name); }
  template <typename... A> Range(const char* fmt, A... a) {
    char buf[128];
    std::snprintf(buf, sizeof buf, fmt, a...);
    roctxRangePushA(buf);
  }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

}  // namespace hdd
