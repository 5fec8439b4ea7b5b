// Device-side body of the FP64 MFMA GEMM tile (see gemm.h), used by the
// single and the batched GEMM kernels; the caller owns the LDS staging.
//
// Block tile 64x64x16, 256 threads = 4 waves in a 2x2 arrangement, each wave
// owning a 32x32 sub-tile made of 2x2 v_mfma_f64_16x16x4 blocks.  Complex
// products use four real MFMAs per block (re*re - im*im, re*im + im*re) on
// interleaved {re, im} operands.
//
// MFMA f64 16x16x4 operand layout (lane l of the wave):
//   A[i][k]: i = l % 16, k = l / 16;  B[k][j]: j = l % 16, k = l / 16;
//   D[i][j] (4 values per lane): j = l % 16, i = l / 16 + 4 * v
// (checked on gfx950 with one-hot inputs; the f32/bf16 forms differ).
#pragma once
#include "common.h"
#include "gemm.h"

namespace psd {
namespace gemmdev {
constexpr int BM = 64, BN = 64, BK = 16, PAD = 4, NT = 256;

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double zero_of(double) { return 0.0; }
__device__ __forceinline__ cd zero_of(cd) { return cmk(0.0, 0.0); }
__device__ __forceinline__ double conj_of(double v) { return v; }
__device__ __forceinline__ cd conj_of(cd v) { return cconj(v); }
__device__ __forceinline__ double scale_of(double v, double s) { return v * s; }
__device__ __forceinline__ cd scale_of(cd v, double s) { return cscale(v, s); }

// The stored element behind op(X)[r][c] (not yet conjugated for OP_C),
// where for A (r, c) = (i, k) and for B (r, c) = (k, j).  `kdim` tells
// which of r/c is the K index (0: r, 1: c).
template <typename T, int OP, int KDIM>
__device__ __forceinline__ T op_raw(const GemmOperand &o, int r, int c) {
    const int k = KDIM == 0 ? r : c;
    const bool second = k >= o.ksplit;
    const T *p = static_cast<const T *>(second ? o.p1 : o.p0);
    const int64_t ld = second ? o.ld1 : o.ld0;
    const int kk = second ? k - o.ksplit : k;
    const int rr = KDIM == 0 ? kk : r, cc = KDIM == 0 ? c : kk;
    return (OP == OP_N) ? p[rr + (int64_t)cc * ld] : p[cc + (int64_t)rr * ld];
}

__device__ __forceinline__ double gamma_dk(double a, double b) {
    const bool pa = a > 0.0, pb = b > 0.0;
    if (pa && pb) return 1.0;
    if (!pa && !pb) return 0.0;
    return pa ? a / (a - b) : b / (b - a);
}

// LDS staging of one k-step: the A and B panels, k-major.
template <typename T>
struct GemmLds {
    T As[BK][BM + PAD];
    T Bs[BK][BN + PAD];
};

// One k-slice of op(A) (rows i0.., BK columns from k0) and of op(B) (BK
// rows from k0, columns j0..) into four registers per thread, zero outside
// the problem; the matching stores put them in the LDS tiles As[k][i],
// Bs[k][j].  The thread-to-element maps keep global reads coalesced.  The
// loads only fetch, at indices clamped into the problem (M, N, K >= 1 where
// they run), every element unconditionally, with the k-scales of A and a
// mask of the elements inside the problem; the zeroing outside it, the
// conjugation and the scaling are applied by the stores, one k-slice later.
// No load then waits where it is issued (a load under a branch, or one
// whose value is used at once, waits for its round trip there).
struct KSlice {
    double ks[4];
    unsigned ok;
};

template <typename T, int OPA>
__device__ __forceinline__ void gemm_load_a(const GemmDesc &d, int i0, int k0, T (&v)[4], KSlice &m) {
    const int t = threadIdx.x;
    m.ok = 0u;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int i = OPA == OP_N ? (t & 63) : (t >> 4) + 16 * s;
        const int k = OPA == OP_N ? (t >> 6) + 4 * s : (t & 15);
        const bool in = i0 + i < d.M && k0 + k < d.K;
        const int ic = min(i0 + i, d.M - 1), kc = min(k0 + k, d.K - 1);
        v[s] = op_raw<T, OPA, 1>(d.A, ic, kc);
        m.ks[s] = d.A.kscale ? d.A.kscale[kc] : 1.0;
        m.ok |= in ? 1u << s : 0u;
    }
}

template <typename T, int OPA>
__device__ __forceinline__ void gemm_store_a(const GemmDesc &d, T (&As)[BK][BM + PAD], const T (&v)[4],
                                             const KSlice &m) {
    const int t = threadIdx.x;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int i = OPA == OP_N ? (t & 63) : (t >> 4) + 16 * s;
        const int k = OPA == OP_N ? (t >> 6) + 4 * s : (t & 15);
        const bool in = (m.ok >> s) & 1u;
        T x = v[s];
        if (OPA == OP_C) x = conj_of(x);
        if (d.A.kscale) x = scale_of(x, m.ks[s]);
        As[k][i] = in ? x : zero_of(T());
    }
}

template <typename T, int OPB>
__device__ __forceinline__ void gemm_load_b(const GemmDesc &d, int j0, int k0, T (&v)[4], unsigned &ok) {
    const int t = threadIdx.x;
    ok = 0u;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int j = OPB == OP_N ? (t >> 4) + 16 * s : (t & 63);
        const int k = OPB == OP_N ? (t & 15) : (t >> 6) + 4 * s;
        const bool in = j0 + j < d.N && k0 + k < d.K;
        v[s] = op_raw<T, OPB, 0>(d.B, min(k0 + k, d.K - 1), min(j0 + j, d.N - 1));
        ok |= in ? 1u << s : 0u;
    }
}

template <typename T, int OPB>
__device__ __forceinline__ void gemm_store_b(T (&Bs)[BK][BN + PAD], const T (&v)[4], unsigned ok) {
    const int t = threadIdx.x;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int j = OPB == OP_N ? (t >> 4) + 16 * s : (t & 63);
        const int k = OPB == OP_N ? (t & 15) : (t >> 6) + 4 * s;
        const bool in = (ok >> s) & 1u;
        T x = v[s];
        if (OPB == OP_C) x = conj_of(x);
        Bs[k][j] = in ? x : zero_of(T());
    }
}

template <typename T, int OPA, int OPB, int EPI>
__device__ void gemm_tile(const GemmDesc &dd, int ti, int tj, int tz, GemmLds<T> &L) {
    auto &As = L.As;
    auto &Bs = L.Bs;
    GemmDesc d = dd;
    if (d.dN) d.N = min(d.N, *d.dN);
    if (d.dK) d.K = min(d.K, *d.dK);
    const int i0 = ti * BM, j0 = tj * BN;
    if (i0 >= d.M || j0 >= d.N) return;
    if (d.lower_only && i0 + BM - 1 < j0) return;
    int kbeg = 0;
    if (d.kchunk > 0) {
        kbeg = tz * d.kchunk;
        d.K = min(d.K, kbeg + d.kchunk);
        d.C = static_cast<void *>(static_cast<char *>(d.C) + (int64_t)tz * d.c_zstride * sizeof(T));
    }
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w & 1, wn = w >> 1;
    constexpr bool CPLX = sizeof(T) == 16;

    v4d acc_r[2][2], acc_i[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            acc_r[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
            acc_i[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
        }

    // The next k-slice is loaded into registers while the current one feeds
    // the MFMAs, then stored to LDS: global latency overlaps the products.
    T av[4], bv[4];
    KSlice am;
    unsigned bok;
    if (kbeg < d.K) {  // (a split-K slice past a device-side K has no products)
        gemm_load_a<T, OPA>(d, i0, kbeg, av, am);
        gemm_load_b<T, OPB>(d, j0, kbeg, bv, bok);
    }
    for (int k0 = kbeg; k0 < d.K; k0 += BK) {
        gemm_store_a<T, OPA>(d, As, av, am);
        gemm_store_b<T, OPB>(Bs, bv, bok);
        __syncthreads();
        if (k0 + BK < d.K) {
            gemm_load_a<T, OPA>(d, i0, k0 + BK, av, am);
            gemm_load_b<T, OPB>(d, j0, k0 + BK, bv, bok);
        }
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            const int kr = ks + (lane >> 4), ii = lane & 15;
            T af[2], bf[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) af[a] = As[kr][wm * 32 + a * 16 + ii];
#pragma unroll
            for (int b = 0; b < 2; ++b) bf[b] = Bs[kr][wn * 32 + b * 16 + ii];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    if constexpr (CPLX) {
                        const cd x = *reinterpret_cast<const cd *>(&af[a]);
                        const cd y = *reinterpret_cast<const cd *>(&bf[b]);
                        acc_r[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, y.x, acc_r[a][b], 0, 0, 0);
                        acc_r[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-x.y, y.y, acc_r[a][b], 0, 0, 0);
                        acc_i[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, y.y, acc_i[a][b], 0, 0, 0);
                        acc_i[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, y.x, acc_i[a][b], 0, 0, 0);
                    } else {
                        const double x = *reinterpret_cast<const double *>(&af[a]);
                        const double y = *reinterpret_cast<const double *>(&bf[b]);
                        acc_r[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc_r[a][b], 0, 0, 0);
                    }
                }
        }
        __syncthreads();
    }

    // ---- epilogue
    const double rt2 = 1.41421356237309504880;
    // C for beta != 0: every value this thread adds to is loaded before the
    // first store (a load placed after a store to the same array would wait
    // for that store, one memory round trip per element)
    T cold[2][2][4];
    if constexpr (EPI != EPI_SVEC) {
        if (d.beta != 0.0 && !(CPLX && d.mirror)) {
            const T *C = static_cast<const T *>(d.C);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = i0 + wm * 32 + a * 16 + (lane >> 4) + 4 * v;
                        const int j = j0 + wn * 32 + b * 16 + (lane & 15);
                        if (i < d.M && j < d.N) cold[a][b][v] = C[i + (int64_t)j * d.ldc];
                    }
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + wm * 32 + a * 16 + (lane >> 4) + 4 * v;
                const int j = j0 + wn * 32 + b * 16 + (lane & 15);
                if (i >= d.M || j >= d.N) continue;
                double re = acc_r[a][b][v], im = CPLX ? acc_i[a][b][v] : 0.0;
                if (EPI == EPI_SVEC) {
                    if (i < j) continue;
                    if (d.dstatus && *d.dstatus == ST_ENONFINITE) re = im = __builtin_nan("");
                    const int64_t n = d.svec_n;
                    const double sgn = d.dsign ? *d.dsign : d.sign;
                    const double *xb = (d.dsign && sgn > 0.0) ? nullptr : d.xbase;
                    const double xs = d.xscale != 0.0 ? d.xscale : 1.0;
                    if (i == j) {
                        const int64_t o = svec_col_start((int)n, j);
                        const double base = xb ? xs * xb[o] : 0.0;
                        d.y[o] = base + sgn * re;
                    } else {
                        const int64_t o = svec_off((int)n, i, j);
                        const double b0 = xb ? xs * xb[o] : 0.0, b1 = xb ? xs * xb[o + 1] : 0.0;
                        d.y[o] = b0 + sgn * rt2 * re;
                        d.y[o + 1] = b1 + sgn * rt2 * im;
                    }
                    continue;
                }
                if (EPI == EPI_GAMMA) {
                    const double g = gamma_dk(d.lam[i], d.lam[j]);
                    re *= g; im *= g;
                }
                T *C = static_cast<T *>(d.C);
                const int64_t idx = i + (int64_t)j * d.ldc;
                if constexpr (CPLX) {
                    cd out = cmk(d.alpha * re + (i == j ? d.diag_add : 0.0), d.alpha * im);
                    if (d.mirror) {
                        if (i < j) continue;  // written as the mirror of (j, i)
                        if (i == j) out.y = 0.0;
                        *reinterpret_cast<cd *>(&C[idx]) = out;
                        if (i != j) *reinterpret_cast<cd *>(&C[j + (int64_t)i * d.ldc]) = cconj(out);
                        continue;
                    }
                    if (d.beta != 0.0) {
                        const cd c0 = *reinterpret_cast<const cd *>(&cold[a][b][v]);
                        out = cmk(out.x + d.beta * c0.x, out.y + d.beta * c0.y);
                    }
                    *reinterpret_cast<cd *>(&C[idx]) = out;
                } else {
                    double out = d.alpha * re + (i == j ? d.diag_add : 0.0);
                    if (d.beta != 0.0) out += d.beta * *reinterpret_cast<const double *>(&cold[a][b][v]);
                    *reinterpret_cast<double *>(&C[idx]) = out;
                }
            }
}

}  // namespace gemmdev
}  // namespace psd
