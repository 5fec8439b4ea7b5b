// FP64 MFMA GEMM used by every dense stage of the large-block path:
//   C = alpha * op(A) op(B) + beta * C      (complex or real, column-major)
// with op in {N, C (conjugate transpose; plain transpose for real data)}.
//
// Operands may be split along K into two parts (p0 for k < ksplit, p1 for
// k >= ksplit): the Hermitian rank-2k update  A -= V W^H + W V^H  is one
// GEMM with A = [V W], B = [W V]^H.  An operand may also carry a per-k real
// scale (columns of op(A) scaled by s[k]), which builds V diag(lambda) on
// the fly for the reconstruction.
//
// Epilogues: plain store; svec pack of the lower triangle (the output is the
// projection, written straight into the caller's svec); Daleckii-Krein
// weights Gamma(lambda_i, lambda_j) applied to the product before the store.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psd {

enum : int { OP_N = 0, OP_C = 1 };
enum : int { EPI_STORE = 0, EPI_SVEC = 1, EPI_GAMMA = 2 };

struct GemmOperand {
    const void *p0;   // part used for k < ksplit
    const void *p1;   // part used for k >= ksplit (may equal p0 with ksplit = K)
    int64_t ld0, ld1; // leading dimensions (elements)
    int ksplit;
    int op;           // OP_N or OP_C
    const double *kscale;  // optional per-k scale (A only)
};

struct GemmDesc {
    int M, N, K;
    int lower_only;   // skip tiles strictly above the diagonal
    GemmOperand A, B;
    void *C;
    int64_t ldc;
    double alpha, beta;
    // EPI_SVEC: y (svec of order N == M), x base (nullable), sign
    double *y;
    const double *xbase;
    int64_t svec_n;
    double sign;
    // EPI_GAMMA: eigenvalues for rows / columns
    const double *lam;
    // Sizes known only on the device: N = min(N, *dN), K = min(K, *dK).
    const int *dN;
    const int *dK;
    // EPI_SVEC: sign read from the device (base x used iff sign < 0).
    const double *dsign;
    // EPI_SVEC: status word of the problem (nullable); when it reports a
    // non-finite input every output entry is NaN.
    const int *dstatus;
    // Split-K: blockIdx.z handles K range [z*kchunk, (z+1)*kchunk) and
    // writes its partial product to C + z*c_zstride (beta must be 0).
    int kchunk;
    int64_t c_zstride;
    // EPI_STORE: out = alpha*acc + beta*C + diag_add*delta_ij
    double diag_add;
    // EPI_SVEC: y = xscale*x + sign*acc (0 means 1, the default)
    double xscale;
    // EPI_STORE of a Hermitian product (complex, lower_only, beta = 0): each
    // lower entry is written with its conjugate mirror, diagonal imaginary
    // parts zero, so the stored result is exactly Hermitian
    int mirror;
    // Lockstep group of nmem problems (0 or 1: a single one): problem b uses
    // every pointer above moved by b * zs bytes, except y and xbase, which
    // move by ioff[b] elements (ioff null: not at all).
    int nmem;
    int64_t zs;
    const int64_t *ioff;
    // Nullable device flag read by every workgroup first: nonzero skips the
    // whole product (a step whose outcome the device decided to drop).
    const int *skip;
};

// Launch one GEMM described by `d` (grid sized from d) on stream st.
hipError_t gemm_launch(const GemmDesc &d, bool complex_data, int epilogue, hipStream_t st);
// Number of split-K slices gemm_launch uses for `d` (1 without kchunk).
__host__ __device__ inline int gemm_kslices(const GemmDesc &d) {
    return d.kchunk > 0 ? (d.K + d.kchunk - 1) / d.kchunk : 1;
}
// Launch `count` GEMMs whose descriptors live in device memory; every one
// has M <= maxM, N <= maxN (grid sized from those bounds).
// With nmem > 1 the descriptors of member b sit b * zs bytes after ddesc.
hipError_t gemm_launch_batched(const GemmDesc *ddesc, int count, int maxM, int maxN, bool complex_data,
                               hipStream_t st, int nmem = 1, int64_t zs = 0);

}  // namespace psd
