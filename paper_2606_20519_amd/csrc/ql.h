// Implicit-shift QL iteration for a real symmetric tridiagonal matrix, run by
// one workgroup on LDS arrays.  Used by the whole-block kernel (order <= 64)
// and by the leaves of the divide-and-conquer tridiagonal eigensolver.
#pragma once
#include "common.h"

namespace psd {

// On entry d[0..n) is the diagonal and e[0..n-1) the off-diagonal of T,
// Z (column-major, leading dimension ldz, rows/cols 0..n) holds the matrix
// the rotations are accumulated into (the identity for T's eigenvectors).
// On exit d holds the eigenvalues (unsorted) and Z <- Z * (rotations), so
// that T = Z diag(d) Z^T when Z started as I.
//
// Each sweep is the implicit QL step of Dubrulle, Martin and Wilkinson
// ("The implicit QL algorithm", Numer. Math. 12, 1968; EISPACK's imtql2): a
// Wilkinson-type shift from the leading 2x2 of the unreduced block, then
// plane rotations chased from its bottom to its top, the shift entering
// only through the first rotation.  Thread 0 computes
// a sweep's rotations sequentially (recording them in rc/rs/ri, >= n
// entries each); then every thread applies them, in order, to its own rows
// of Z.  nrot/done are LDS scalars.  All threads must call this.
// Returns ST_OK or ST_ENOCONV (more than 60 sweeps for one eigenvalue).
__device__ inline int ql_implicit(double *d, double *e, double *Z, int ldz, int n, double *rc,
                                  double *rs, int *ri, int *nrot_s, int *done_s) {
    const int t = threadIdx.x;
    const double eps = 2.220446049250313e-16;
    int l = 0, iter = 0, status = ST_OK;  // meaningful in thread 0 only
    if (t == 0) { e[n - 1] = 0.0; *done_s = 0; }
    __syncthreads();
    while (true) {
        if (t == 0) {
            int nrot = 0;
            while (l < n) {
                int m = l;
                for (; m < n - 1; ++m) {
                    const double dd = fabs(d[m]) + fabs(d[m + 1]);
                    if (fabs(e[m]) <= eps * dd) break;
                }
                if (m == l) { ++l; iter = 0; continue; }
                if (++iter > 60) { status = ST_ENOCONV; l = n; break; }
                double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                double r = hypot(g, 1.0);
                g = d[m] - d[l] + e[l] / (g + copysign(r, g));
                double s = 1.0, c = 1.0, p = 0.0;
                int i = m - 1;
                bool early = false;
                for (; i >= l; --i) {
                    const double f = s * e[i], b = c * e[i];
                    r = hypot(f, g);
                    e[i + 1] = r;
                    if (r == 0.0) { d[i + 1] -= p; e[m] = 0.0; early = true; break; }
                    s = f / r; c = g / r;
                    g = d[i + 1] - p;
                    r = (d[i] - g) * s + 2.0 * c * b;
                    p = s * r;
                    d[i + 1] = g + p;
                    g = c * r - b;
                    rc[nrot] = c; rs[nrot] = s; ri[nrot] = i;
                    ++nrot;
                }
                if (!early) { d[l] -= p; e[l] = g; e[m] = 0.0; }
                break;  // one sweep produced: let everybody apply it
            }
            *nrot_s = nrot;
            *done_s = (l >= n);
        }
        __syncthreads();
        const int nrot = *nrot_s;
        for (int row = t; row < n; row += blockDim.x) {
            for (int k = 0; k < nrot; ++k) {
                const int i = ri[k];
                const double c = rc[k], s = rs[k];
                const double zi = Z[row + i * ldz], zi1 = Z[row + (i + 1) * ldz];
                Z[row + (i + 1) * ldz] = s * zi + c * zi1;
                Z[row + i * ldz] = c * zi - s * zi1;
            }
        }
        const int done = *done_s;
        __syncthreads();
        if (done) break;
    }
    // broadcast the status of thread 0
    if (t == 0) *nrot_s = status;
    __syncthreads();
    const int st = *nrot_s;
    __syncthreads();
    return st;
}

}  // namespace psd
