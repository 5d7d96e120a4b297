// Optional per-kernel timing with HIP events recorded on the launch stream.
#pragma once
#include <hip/hip_runtime.h>

namespace spike {

bool prof_enabled();
int prof_begin(const char* name, hipStream_t st);   // returns a slot (or -1)
void prof_end(int slot, hipStream_t st);

// Records a start event at construction and an end event at destruction
// around one kernel launch, when profiling is enabled.
struct ProfScope {
  int slot;
  hipStream_t st;
  ProfScope(const char* name, hipStream_t s) : slot(-1), st(s) {
    if (prof_enabled()) slot = prof_begin(name, s);
  }
  ~ProfScope() {
    if (slot >= 0) prof_end(slot, st);
  }
};

}  // namespace spike
