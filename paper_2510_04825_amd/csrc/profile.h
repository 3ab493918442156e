// Per-kernel timing with HIP events.  When enabled (subap_profile_enable),
// every kernel launch site wrapped in a ProfScope records an event pair on
// its stream; subap_profile_entry synchronizes on the recorded events and
// reports per-name call counts and total milliseconds.
#pragma once

#include <hip/hip_runtime.h>

namespace subap {

bool profiling_enabled();
void profile_push(const char* name, hipEvent_t a, hipEvent_t b);
hipEvent_t profile_event();

class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t st) : name_(name), st_(st) {
    // no events inside a graph capture: the launch is recorded, not run
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (profiling_enabled() && hipStreamIsCapturing(st_, &cap) == hipSuccess &&
        cap == hipStreamCaptureStatusNone) {
      a_ = profile_event();
      if (a_) (void)hipEventRecord(a_, st_);
    }
  }
  ~ProfScope() {
    if (a_) {
      hipEvent_t b = profile_event();
      if (b) {
        (void)hipEventRecord(b, st_);
        profile_push(name_, a_, b);
      }
    }
  }
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  const char* name_;
  hipStream_t st_;
  hipEvent_t a_ = nullptr;
};

}  // namespace subap
