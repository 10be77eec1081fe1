// Opt-in per-kernel-class timing: hipEvents recorded around each launch on
// the launch's stream, plus the algorithmic flops and bytes of the launch.
#pragma once

#include "common.hpp"

namespace msqrt {

bool prof_enabled();
// Returns a token (>= 0) or -1 when profiling is off.
int prof_begin(hipStream_t st);
// Destroys the cached timing events (pending ones are resolved first).
void prof_release();
void prof_end(int token, hipStream_t st, const char* cls, double flops, double bytes);

}  // namespace msqrt
