// Optional device timing of individual kernel launches (mk_profile_*).
#pragma once

#include <hip/hip_runtime.h>

namespace mk {

bool profiling_enabled();

// Records a HIP event on `stream` when constructed and another when destroyed
// (if profiling is enabled), attributing the interval to `name`.
class ProfScope {
  public:
    ProfScope(const char* name, hipStream_t stream);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;

  private:
    const char* name_;
    hipStream_t stream_;
    hipEvent_t start_ = nullptr;
};

}  // namespace mk
