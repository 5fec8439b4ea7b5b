// Optional launch timing (psd_timing_start / psd_timing_stop).
#pragma once
#include <hip/hip_runtime.h>

namespace psd {

enum { KF_HEMV = 1, KF_GEMM = 2, KF_NS = 3, KF_WSTEP = 4 };

// Records the start event of a timed launch of `family` on `st`; returns the
// slot to close with timing_end, or -1 if this launch is not timed.
int timing_begin(int family, hipStream_t st);
void timing_end(int slot, hipStream_t st, double work);

}  // namespace psd
