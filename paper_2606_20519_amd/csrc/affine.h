// Internal batched forms of the affine step and the constraint maps
// (affine.hip), used by the SCS solver to cover a batch of instances with
// one launch per pass: instance z's vectors sit xs / ys elements after
// instance 0's, its two workspace tensors wss bytes after instance 0's
// workspace (psd_affine_workspace_size bytes each).  An instance whose flag
// in `active` (device int[nb], nullable) is 0 is left untouched.  No
// validation: the caller has checked d, alignment and sizes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psd {

// (zx, zy) = ((ax - A^T ay)/2, ay + A zx); zx may alias ax, zy may alias ay.
hipError_t affine_step_batched(int d, const double *ax, const double *ay, double *zx, double *zy, int64_t xs,
                               int64_t ys, void *ws, int64_t wss, int nb, const int *active, hipStream_t st);
// y = A x.
hipError_t constraint_apply_batched(int d, const double *x, double *y, int64_t xs, int64_t ys, void *ws, int64_t wss,
                                    int nb, const int *active, hipStream_t st);
// x = A^T y.
hipError_t constraint_adjoint_batched(int d, const double *y, double *x, int64_t ys, int64_t xs, void *ws,
                                      int64_t wss, int nb, const int *active, hipStream_t st);

}  // namespace psd
