// Warm-started FP64 projection (warm.hip): refinement of a nearby
// eigen-pair by matrix products, with the cold path as the host's fallback.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "kernels.h"

namespace psd {

constexpr int WARM_STEPS = 5;          // refinement steps at most
constexpr double WARM_STOP = 1e-7;     // max |E_ij| after which the next step is skipped
constexpr double WARM_ACCEPT = 1e-6;   // max |E_ij| of the last step for the result to stand
constexpr double WARM_GIVE_UP = 0.5;   // a step above this (or above half the previous) ends the attempt

// device flags (ints) and scalars (doubles) of one refinement
enum : int { WF_STATUS = 0, WF_ITERS = 1, WF_REJECT = 2, WF_SKIP = 3, WF_COUNT = WF_SKIP + WARM_STEPS + 1 };
enum : int { WS_LMAX = 0, WS_ELAST = 1 };

struct WarmWs {
    int n;
    int64_t ld;        // leading dimension of every matrix (= n)
    int ksf, kcf;      // split-K slices of the full products (A X, X E) and rows per slice
    int ksl, kcl;      // the same for the lower-tile products (X^H B, X^H X)
    double2 *A;        // the input, full Hermitian (M = conj X)
    double2 *X[2];     // eigenvector estimates, ping-pong
    double2 *B;        // A X
    double2 *E;        // correction
    double2 *P1, *P2;  // split-K partials (ks slices each)
    double *lam;       // Rayleigh quotients
    double *lamp;      // max(lambda, 0)
    int npairs;        // lower tile pairs of the correction pass
    double *epart;     // per-pair max |E_ij|^2
    double *scal;      // WS_* scalars
    int *flags;        // WF_* flags
};

// Bytes of the refinement workspace of order n; carves it when base is non-null.
size_t warm_layout(int n, void *base, WarmWs *w);
// Enqueues the refinement of saved_prev's eigenvectors for x, the
// reconstruction into y and (when non-null) the refined pair into
// saved_out; the last two only when the result is accepted, which
// w.flags[WF_REJECT] == 0 reports once the stream reaches it.
hipError_t warm_refine(const WarmWs &w, const double *x, const double *saved_prev, double *y, double *saved_out,
                       psd_dev_info *info, hipStream_t st);

}  // namespace psd
