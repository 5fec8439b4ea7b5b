// Internal launch interface between the host runtime (abi.hip) and the
// kernels.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace psd {

// Same layout as the public psd_info.
struct psd_dev_info {
    int32_t status, n_pos, n_neg, iters, fallback, reserved;
    double est_rel_err;
    double scale;
};

// One small block (order <= 64) for the whole-block LDS kernel.
struct SmallJob {
    int64_t offset;        // svec offset of the block in x / y
    int64_t saved_offset;  // offset of its saved record (doubles), if saving
    int32_t n;
    int32_t info_index;
};

size_t small_lds_bytes();
// One-time kernel attribute setup (dynamic LDS limits); call outside graph capture.
hipError_t small_prepare();
hipError_t dc_prepare();
// Workgroup size the order-<= 32 kernel needs for a block of order n.
int small32_threads(int n);
// jobs[0 .. n32) have order <= 32 (the one-barrier-per-step kernel, run
// with nt32 threads: the largest small32_threads of their orders), the rest
// order 33 .. 64.
hipError_t launch_small(const SmallJob *jobs, int njobs, int n32, int nt32, const double *x, double *y,
                        psd_dev_info *infos, double *saved, hipStream_t st);
hipError_t launch_small_one(const SmallJob &job, const double *x, double *y, psd_dev_info *info,
                            double *saved, hipStream_t st);

}  // namespace psd
