// Optional stage timing with HIP events on the caller's stream (off by default).
#pragma once

#include <hip/hip_runtime.h>

namespace skew {

struct StageTimer {
  int slot = -1;  // -1: timing off
};

// Record the start of stage `name` on stream s (no-op while timing is off).
StageTimer stage_begin(const char *name, hipStream_t s);
// Record the end of the stage.
void stage_end(const StageTimer &t, hipStream_t s);

}  // namespace skew
