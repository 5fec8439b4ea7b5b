// Workspace and launcher of the mixed-precision Newton-Schulz projection.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "kernels.h"

namespace psd {

struct MixedWs {
    int n;
    int64_t lda;        // FP64 matrices (complex, column-major)
    int npad;           // low-precision planes: npad x npad, npad % 64 == 0
    double2 *M, *S, *S2, *T64;
    void *lo0, *lo1, *lo2;   // two planes (re, im) each
    double2 *q, *qprev, *wv, *P;
    double *ab, *alpha, *red;
    float *part;        // split partial sums of the BF16 128x128 product (large npad)
    int ns_big;         // npad from which the BF16 product uses 128x128 tiles
    int *status;
    // lockstep group (as for the FP64 path: member b uses the slot b * zs
    // bytes on, svec offset ioff[b], info record infoidx[b]); single block:
    // nmem = 1, zs = 0, null tables
    int nmem;
    int64_t zs;
    const int64_t *ioff;
    const int *infoidx;
};

// The BF16 Newton-Schulz product takes 128x128 tiles from this npad on (64x64
// below): the default of single calls and eager groups; a plan may lower it
// to NS_BIG_MIN (its autotuner times both).  Below 2048 the 128x128 form
// never splits its tail, so the workspace is the same either way.
constexpr int NS_BIG_DEFAULT = 2048;
constexpr int NS_BIG_MIN = 1024;

// mode: 1 = BF16, 2 = FP32, 3 = split BF16 (hi + lo, three products per real
// product) low-precision iterations.
size_t mixed_layout(int n, int mode, void *base, MixedWs *w);
hipError_t mixed_project(const MixedWs &w, int mode, const double *x, double *y, psd_dev_info *info, int iters,
                         int corr, hipStream_t st);

}  // namespace psd
