// Mixed-precision projection by the Newton-Schulz sign iteration.
//
// Pi(X) = (X + X sign(X)) / 2, because max(t, 0) = (t + t sgn t)/2 on each
// eigenvalue.  sign(X) is the limit of X_{k+1} = X_k (3I - X_k^2)/2 from
// X_0 = X/alpha with alpha >= ||X||_2 (the cubic converges to sgn t for
// |t| < sqrt3): a composite matrix polynomial built from matrix products only,
// the kind of factorisation-free projection the paper's outlook proposes
// (Sec. V, "Approximate semidefinite-cone projections").
//
// Stages (FP64 only where it buys accuracy):
//  * scale: alpha from a short FP64 Lanczos run (24 Hermitian mat-vecs, then
//    the extreme eigenvalues of the small tridiagonal by Sturm-count
//    multisection), alpha = 1.1 max|theta|;
//  * X_0 = X/alpha rounded (RNE) to BF16 or FP32 planar complex;
//  * K scaled iterations X_{k+1} = (a_k/2) X_k (3I - a_k^2 X_k^2) (Chen and
//    Chow's scaled Newton-Schulz, scalings capped at 1.5: a_k from the known
//    bound on the spectrum, 21 steps instead of 40 for the same resolution),
//    each two complex GEMMs
//    on the MFMA cores with FP32 accumulation: T = 3I - a_k^2 X_k^2, then
//    X_{k+1} = (a_k/2) X_k T (scalings in the epilogues); the last product is
//    kept in FP64;
//  * c FP64 correction steps S <- S (3I - S^2)/2 (FP64 MFMA GEMMs over the
//    lower tiles, each written with its conjugate mirror: both products are
//    Hermitian), which square the error of every eigenvalue of S whose sign
//    the low-precision iterations already resolved;
//  * F = X S by one full FP64 GEMM, then Pi = X/2 + (F + F^H)/4, the
//    Hermitian part (X and the exact sign commute), written as the svec;
//    the anti-Hermitian part F - F^H = [X, S] and ||X||_F^2 - ||F||_F^2
//    give the error estimate, and n_pos comes from tr S.
// The low-precision iterations return the sign of a matrix within about
// K u ||X|| of X (u = 2^-8 for BF16, 2^-24 for FP32); since Pi is
// 1-Lipschitz the result is within that distance of Pi(X), and components
// with |lambda| below it may be classified either way.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "large.h"
#include "mixed.h"
#include "timing.h"

namespace psd {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef short v8s __attribute__((ext_vector_type(8)));

constexpr int LZ_STEPS = 24;
constexpr int LZ_SPLIT = 16;  // column splits of the Lanczos mat-vec

// Counter-based pseudo-random value in [-0.5, 0.5) (splitmix64).
__device__ inline double hash_unit(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return (double)(x >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

__global__ void __launch_bounds__(1024) lz_init_kernel(int n, double2 *q, double2 *qprev, double *ab, int64_t zs) {
    __shared__ double red[32];
    q = member_ptr(q, zs, blockIdx.z);
    qprev = member_ptr(qprev, zs, blockIdx.z);
    ab = member_ptr(ab, zs, blockIdx.z);
    double part = 0.0;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        const double2 v = cmk(hash_unit(2 * (uint64_t)r), hash_unit(2 * (uint64_t)r + 1));
        q[r] = v;
        qprev[r] = cmk(0.0, 0.0);
        part += cabs2(v);
    }
    const double inv = 1.0 / sqrt(block_sum(part, red));
    for (int r = threadIdx.x; r < n; r += blockDim.x) q[r] = cscale(q[r], inv);
    if (threadIdx.x < 2 * LZ_STEPS + 4) ab[threadIdx.x] = 0.0;
}

// P[cs][row] = sum over the column chunk cs of M(row, col) q(col).
__global__ void __launch_bounds__(256) lz_gemv_kernel(const double2 *__restrict__ M, int64_t lda, int n,
                                                      const double2 *__restrict__ q, double2 *P, int64_t zs) {
    __shared__ double2 part[4][64];
    M = member_ptr(M, zs, blockIdx.z);
    q = member_ptr(q, zs, blockIdx.z);
    P = member_ptr(P, zs, blockIdx.z);
    const int rb = blockIdx.x, cs = blockIdx.y, t = threadIdx.x, r = t & 63, g = t >> 6;
    const int row = rb * 64 + r;
    const int chunk = (n + LZ_SPLIT - 1) / LZ_SPLIT;
    const int c0 = cs * chunk, c1 = min(n, c0 + chunk);
    double2 acc = cmk(0.0, 0.0);
    if (row < n) {
#pragma unroll 4
        for (int c = c0 + g; c < c1; c += 4) acc = cfma(M[row + (int64_t)c * lda], q[c], acc);
    }
    part[g][r] = acc;
    __syncthreads();
    if (t < 64 && row < n)
        P[(int64_t)cs * n + row] = cadd(cadd(part[0][t], part[1][t]), cadd(part[2][t], part[3][t]));
}

// One Lanczos step on a single workgroup: y = sum P, a = Re q^H y,
// w = y - a q - b_prev q_prev, b = ||w||, (q_prev, q) <- (q, w / b).
__global__ void __launch_bounds__(1024) lz_step_kernel(int n, int step, const double2 *__restrict__ P, double2 *q,
                                                       double2 *qprev, double2 *wv, double *ab, int64_t zs) {
    __shared__ double red[32];
    P = member_ptr(P, zs, blockIdx.z);
    q = member_ptr(q, zs, blockIdx.z);
    qprev = member_ptr(qprev, zs, blockIdx.z);
    wv = member_ptr(wv, zs, blockIdx.z);
    ab = member_ptr(ab, zs, blockIdx.z);
    if (ab[2 * LZ_STEPS + 2] != 0.0) return;  // broke down earlier
    double part = 0.0;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        double2 y = cmk(0.0, 0.0);
        for (int cs = 0; cs < LZ_SPLIT; ++cs) y = cadd(y, P[(int64_t)cs * n + r]);
        wv[r] = y;
        part += cmulc(q[r], y).x;
    }
    const double a = block_sum(part, red);
    const double bprev = step > 0 ? ab[LZ_STEPS + step - 1] : 0.0;
    part = 0.0;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        const double2 w = csub(csub(wv[r], cscale(q[r], a)), cscale(qprev[r], bprev));
        wv[r] = w;
        part += cabs2(w);
    }
    const double b = sqrt(block_sum(part, red));
    if (threadIdx.x == 0) {
        ab[step] = a;
        ab[LZ_STEPS + step] = b;
        ab[2 * LZ_STEPS] = step + 1;  // steps done
    }
    const double nrmx = fabs(a) + bprev;
    if (!(b > 1e-14 * nrmx)) {
        if (threadIdx.x == 0) ab[2 * LZ_STEPS + 2] = 1.0;  // invariant subspace: Ritz values exact
        return;
    }
    const double inv = 1.0 / b;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        qprev[r] = q[r];
        q[r] = cscale(wv[r], inv);
    }
}

// alpha = 1.1 max |theta| over the Ritz values of the Lanczos tridiagonal.
// Eigenvalues of the real symmetric tridiagonal (d, e) of order k below x
// (Sturm count: negative pivots of T - xI = L D L^T).
__device__ __forceinline__ int lz_sturm(const double *d, const double *e, int k, double x) {
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < k; ++i) {
        const double off = i > 0 ? e[i - 1] * e[i - 1] / q : 0.0;
        q = d[i] - x - off;
        if (q == 0.0) q = -1e-300;  // a zero pivot counts as negative (x at an eigenvalue)
        cnt += q < 0.0 ? 1 : 0;
    }
    return cnt;
}

// alpha = 1.1 max |theta| over the Ritz values theta of the k-step Lanczos
// tridiagonal: its largest and smallest eigenvalues by multisection, the 64
// lanes testing 64 shifts of the current interval per step (the interval
// shrinks 65-fold), from the Gershgorin bounds until it is below 1e-14 of
// its magnitude; the interval's outer end bounds |theta| from above.
__global__ void __launch_bounds__(64) lz_final_kernel(const double *ab, double *alpha_out, int64_t zs) {
    __shared__ double d[LZ_STEPS], e[LZ_STEPS];
    ab = member_ptr(ab, zs, blockIdx.z);
    alpha_out = member_ptr(alpha_out, zs, blockIdx.z);
    const int k = (int)ab[2 * LZ_STEPS];
    const int t = threadIdx.x;
    if (t < k) { d[t] = ab[t]; e[t] = t < k - 1 ? ab[LZ_STEPS + t] : 0.0; }
    __syncthreads();
    if (k <= 0) {
        if (t == 0) *alpha_out = 1.0;
        return;
    }
    double glo = 0.0, ghi = 0.0;
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < k - 1 ? fabs(e[i]) : 0.0);
        glo = i == 0 ? d[i] - r : fmin(glo, d[i] - r);
        ghi = i == 0 ? d[i] + r : fmax(ghi, d[i] + r);
    }
    double bound[2];
    for (int side = 0; side < 2; ++side) {
        // side 0: largest eigenvalue (count(x) == k iff x > it);
        // side 1: smallest (count(x) >= 1 iff x > it)
        double lo = glo - 1e-300, hi = ghi + 1e-300;
        for (int it = 0; it < 20 && hi - lo > 1e-14 * fmax(fabs(lo), fabs(hi)); ++it) {
            const double x = lo + (hi - lo) * (double)(t + 1) / 65.0;
            const int cnt = lz_sturm(d, e, k, x);
            const bool above = side == 0 ? cnt == k : cnt >= 1;
            // the first lane whose shift lies above the eigenvalue
            const unsigned long long mask = __ballot(above);
            const int first = mask ? __ffsll(mask) - 1 : 64;
            const double nhi = first < 64 ? lo + (hi - lo) * (double)(first + 1) / 65.0 : hi;
            const double nlo = first > 0 ? lo + (hi - lo) * (double)first / 65.0 : lo;
            lo = nlo;
            hi = nhi;
        }
        bound[side] = side == 0 ? hi : lo;
    }
    if (t == 0) {
        const double m = fmax(fabs(bound[0]), fabs(bound[1]));
        *alpha_out = m > 0.0 ? 1.1 * m : 1.0;
    }
}

// Full Hermitian matrix from the svec (M = conj X, see common.h); flags
// non-finite entries.
__global__ void __launch_bounds__(256) mx_unpack_kernel(const double *__restrict__ x, double2 *M, int64_t lda, int n,
                                                        int *status, int64_t zs, const int64_t *__restrict__ ioff) {
    M = member_ptr(M, zs, blockIdx.z);
    status = member_ptr(status, zs, blockIdx.z);
    if (ioff) x += ioff[blockIdx.z];
    const int j = blockIdx.y;
    const int i = j + blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double rs2 = 0.70710678118654752440;
    double2 v;
    if (i == j) {
        v = cmk(x[svec_col_start(n, j)], 0.0);
    } else {
        const int64_t o = svec_off(n, i, j);
        v = cmk(x[o] * rs2, x[o + 1] * rs2);
        M[j + (int64_t)i * lda] = cconj(v);
    }
    if (!(isfinite(v.x) && isfinite(v.y))) status[2] = ST_ENONFINITE;
    M[i + (int64_t)j * lda] = v;
}

__global__ void mx_init_kernel(int *status, int64_t zs) {
    status = member_ptr(status, zs, blockIdx.z);
    if (threadIdx.x < 4) status[threadIdx.x] = 0;
}

template <typename L>
__device__ __forceinline__ L to_low(float v);
template <>
__device__ __forceinline__ __bf16 to_low<__bf16>(float v) { return (__bf16)v; }
template <>
__device__ __forceinline__ float to_low<float>(float v) { return v; }

// X0 = M / alpha in low precision, planar, ld = npad; zero padding.
template <typename L>
__global__ void __launch_bounds__(256) ns_scale_kernel(const double2 *__restrict__ M, int64_t lda, int n, int npad,
                                                       const double *alpha, L *Xre, L *Xim, int64_t zs) {
    M = member_ptr(M, zs, blockIdx.z);
    alpha = member_ptr(alpha, zs, blockIdx.z);
    Xre = member_ptr(Xre, zs, blockIdx.z);
    Xim = member_ptr(Xim, zs, blockIdx.z);
    const int j = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= npad) return;
    const double inv = 1.0 / *alpha;
    double2 v = cmk(0.0, 0.0);
    if (i < n && j < n) v = M[i + (int64_t)j * lda];
    Xre[i + (int64_t)j * npad] = to_low<L>((float)(v.x * inv));
    Xim[i + (int64_t)j * npad] = to_low<L>((float)(v.y * inv));
}

// The two-term BF16 split of an FP32 value: hi = bf16(v), lo = bf16(v - hi)
// (v - hi is exact in FP32), so hi + lo carries about 16 significant bits.
__device__ __forceinline__ void bf16_split(float v, __bf16 &hi, __bf16 &lo) {
    hi = (__bf16)v;
    lo = (__bf16)(v - (float)hi);
}

// X0 = M / alpha as split BF16 planes: Re hi, Im hi at X, X + plane; the lo
// terms lo_off elements further.
__global__ void __launch_bounds__(256) ns_scale_split_kernel(const double2 *__restrict__ M, int64_t lda, int n,
                                                             int npad, const double *alpha, __bf16 *X, int64_t plane,
                                                             int64_t lo_off, int64_t zs) {
    M = member_ptr(M, zs, blockIdx.z);
    alpha = member_ptr(alpha, zs, blockIdx.z);
    X = member_ptr(X, zs, blockIdx.z);
    const int j = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= npad) return;
    const double inv = 1.0 / *alpha;
    double2 v = cmk(0.0, 0.0);
    if (i < n && j < n) v = M[i + (int64_t)j * lda];
    const int64_t o = i + (int64_t)j * npad;
    __bf16 h, l;
    bf16_split((float)(v.x * inv), h, l);
    X[o] = h;
    X[o + lo_off] = l;
    bf16_split((float)(v.y * inv), h, l);
    X[o + plane] = h;
    X[o + plane + lo_off] = l;
}

enum { NS_EPI_T = 0, NS_EPI_HALF = 1, NS_EPI_F64 = 2 };

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2), so workgroup g runs on XCD g % 8.  This maps the workgroups of each
// XCD to a contiguous run of tiles (in the row-major lower-triangle order,
// consecutive tiles share the A panel and nearby B panels), a bijection
// onto 0..T-1: XCD x takes T/8 tiles (one more for x < T % 8).
__device__ __forceinline__ int xcd_tile(int g, int T) {
    const int per = T >> 3, rem = T & 7, x = g & 7, idx = g >> 3;
    return x * per + min(x, rem) + idx;
}

// NQ 16-byte chunks of each plane of A (at ao) and B (at bo).
template <typename L, int NQ>
__device__ __forceinline__ void ns_load_chunks(const L *__restrict__ Are, const L *__restrict__ Aim,
                                               const L *__restrict__ Bre, const L *__restrict__ Bim, int64_t ao,
                                               int64_t bo, uint4 (&xr)[NQ], uint4 (&xi)[NQ], uint4 (&yr)[NQ],
                                               uint4 (&yi)[NQ]) {
    constexpr int E = 16 / (int)sizeof(L);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        xr[q] = *reinterpret_cast<const uint4 *>(Are + ao + q * E);
        xi[q] = *reinterpret_cast<const uint4 *>(Aim + ao + q * E);
        yr[q] = *reinterpret_cast<const uint4 *>(Bre + bo + q * E);
        yi[q] = *reinterpret_cast<const uint4 *>(Bim + bo + q * E);
    }
}

typedef float v16f __attribute__((ext_vector_type(16)));

// Epilogue of one 32x32 block at (ib, jb), BF16 planes (as ns_gemm_kernel's
// 16x16 one: the lower part with its conjugate mirror).  32x32x16 output
// layout: D[i][j] in lane j + 32 ((i / 4) % 2), element 4 (i / 8) + i % 4.
template <int SPLIT = 1>
__device__ __forceinline__ void ns_store_block32(const v16f &accr, const v16f &acci, int ib, int jb, int lane, int npad,
                                                 int epi, float c, __bf16 *Cre, __bf16 *Cim, double2 *C64,
                                                 int64_t ld64, int n, int64_t lo_off = 0) {
    if (ib < jb || ib >= npad) return;
    const int j = jb + (lane & 31), ih = 4 * (lane >> 5);
    if (epi != NS_EPI_F64 && ib > jb) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int ir = ib + 8 * g + ih;
            union { __bf16 h[4]; uint2 u; } pr, pi, pn, qr, qi, qn;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float re = accr[4 * g + v], im = acci[4 * g + v];
                if (epi == NS_EPI_T) { re = -c * re; im = -c * im; }
                else { re *= c; im *= c; }
                if constexpr (SPLIT == 2) {
                    bf16_split(re, pr.h[v], qr.h[v]);
                    bf16_split(im, pi.h[v], qi.h[v]);
                    pn.h[v] = -pi.h[v];
                    qn.h[v] = -qi.h[v];
                } else {
                    pr.h[v] = (__bf16)re;
                    pi.h[v] = (__bf16)im;
                    pn.h[v] = (__bf16)(-im);
                }
            }
            const int64_t o = (int64_t)ir + (int64_t)j * npad;
            *reinterpret_cast<uint2 *>(Cre + o) = pr.u;
            *reinterpret_cast<uint2 *>(Cim + o) = pi.u;
            if constexpr (SPLIT == 2) {
                *reinterpret_cast<uint2 *>(Cre + lo_off + o) = qr.u;
                *reinterpret_cast<uint2 *>(Cim + lo_off + o) = qi.u;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t om = (int64_t)j + (int64_t)(ir + v) * npad;
                Cre[om] = pr.h[v];
                Cim[om] = pn.h[v];
                if constexpr (SPLIT == 2) {
                    Cre[lo_off + om] = qr.h[v];
                    Cim[lo_off + om] = qn.h[v];
                }
            }
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = ib + 8 * (r >> 2) + ih + (r & 3);
        if (i < j) continue;
        float re = accr[r], im = acci[r];
        if (epi == NS_EPI_T) { re = (i == j ? 3.0f : 0.0f) - c * re; im = -c * im; }
        else { re *= c; im *= c; }
        if (i == j) im = 0.0f;
        if (epi != NS_EPI_F64) {
            const int64_t o = (int64_t)i + (int64_t)j * npad, om = (int64_t)j + (int64_t)i * npad;
            if constexpr (SPLIT == 2) {
                __bf16 hr, lr, hi, li;
                bf16_split(re, hr, lr);
                bf16_split(im, hi, li);
                Cre[o] = hr; Cim[o] = hi;
                Cre[om] = hr; Cim[om] = -hi;
                Cre[lo_off + o] = lr; Cim[lo_off + o] = li;
                Cre[lo_off + om] = lr; Cim[lo_off + om] = -li;
            } else {
                const __bf16 lr = (__bf16)re, li = (__bf16)im, lni = (__bf16)(-im);
                Cre[o] = lr; Cim[o] = li;
                Cre[om] = lr; Cim[om] = lni;
            }
        } else if (i < n && j < n) {
            C64[i + (int64_t)j * ld64] = cmk((double)re, (double)im);
            C64[j + (int64_t)i * ld64] = cmk((double)re, -(double)im);
        }
    }
}

// C = A B for Hermitian A, B that commute (polynomials in the same X), so C
// is Hermitian: only the lower tiles (ti >= tj) are computed, and each is
// written together with its conjugate mirror, which keeps every iterate
// exactly Hermitian in storage (diagonal imaginary parts set to zero).  That
// exactness matters: A(i,k) is read as conj(A(k,i)) so that both operands
// stream along k within a column, and for a non-Hermitian iterate this
// would multiply by A^H -- a substitution under which rounding errors that
// anticommute with sign(X) double at every step.
// Planar low precision, column-major, ld npad (npad % 64 == 0), FP32
// accumulation on the MFMA cores.  Tile 64x64x32, 4 waves in 2x2, each
// 32x32 = 2x2 MFMA blocks of 16x16.
// SPLIT = 2 (BF16 only): every operand is the two-term split hi + lo of its
// FP32 value (the lo planes lo_off elements after the hi ones), and each
// real product is formed as hi*hi + hi*lo + lo*hi (the lo*lo term, below
// 2^-16 relative, is dropped): three BF16 MFMAs for about 16 significant
// bits, the split ("BF16x3") products of the paper's outlook (Sec. V).
template <typename L, int SPLIT = 1>
__global__ void __launch_bounds__(256) ns_gemm_kernel(const L *__restrict__ Are, const L *__restrict__ Aim,
                                                      const L *__restrict__ Bre, const L *__restrict__ Bim, int npad,
                                                      int epi, float c, L *Cre, L *Cim, double2 *C64, int64_t ld64,
                                                      int n, int64_t zs, int64_t lo_off = 0) {
    constexpr bool BF = sizeof(L) == 2;
    constexpr bool X3 = SPLIT == 2;
    static_assert(!X3 || BF, "split products are BF16");
    {
        const int mb = blockIdx.z;
        Are = member_ptr(Are, zs, mb);
        Aim = member_ptr(Aim, zs, mb);
        Bre = member_ptr(Bre, zs, mb);
        Bim = member_ptr(Bim, zs, mb);
        Cre = member_ptr(Cre, zs, mb);
        Cim = member_ptr(Cim, zs, mb);
        C64 = member_ptr(C64, zs, mb);
    }
    // LDS rows: BF16 64 bytes unpadded, the 16-byte chunk q of row r at
    // position q ^ f(r), f(r) = ((r >> 2) ^ (r >> 1)) & 3 (conflict-free
    // stores and fragment reads); FP32 padded by 4
    constexpr int KP = 32 + (BF ? 0 : 4);
    constexpr int LR = X3 ? 64 : 1;   // the lo planes' tiles (split products only)
    __shared__ __align__(16) L sAr[64][KP], sAi[64][KP], sBr[64][KP], sBi[64][KP];
    __shared__ __align__(16) L sArl[LR][KP], sAil[LR][KP], sBrl[LR][KP], sBil[LR][KP];
    const int tb = xcd_tile(blockIdx.x, gridDim.x);
    int ti = (int)((sqrt(8.0 * tb + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= tb) ++ti;
    while (ti * (ti + 1) / 2 > tb) --ti;
    const int tj = tb - ti * (ti + 1) / 2;
    const int i0 = ti * 64, j0 = tj * 64;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w & 1, wn = w >> 1;
    // FP32: 2x2 blocks of 16x16x4 per wave; BF16: one 32x32x16 block per wave
    // (two accumulators: with one wave per SIMD, as for a single block of
    // order ~1300, the 32x32 form keeps the MFMA pipe far busier)
    v4f accr[2][2], acci[2][2];
    v16f accr32, acci32;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) { accr[a][b] = v4f{0, 0, 0, 0}; acci[a][b] = v4f{0, 0, 0, 0}; }
#pragma unroll
    for (int r = 0; r < 16; ++r) { accr32[r] = 0.0f; acci32[r] = 0.0f; }
    const bool idle = ti == tj && wm == 0 && wn == 1;  // wave tile above the diagonal
    // loader: thread t covers row (t/4) of the tile, k = 8*(t%4) .. +7.
    // BF16: one 16-byte chunk per plane, and the next k-slice is loaded into
    // registers while the current one feeds the MFMAs.  FP32: loaded per
    // slice (the prefetch spills registers there).
    const int lr = t >> 2, lk = (t & 3) * 8;
    const int lks = BF ? (((t & 3) ^ (((lr >> 2) ^ (lr >> 1)) & 3)) * 8) : lk;  // swizzled store position
    uint4 xr[1], xi[1], yr[1], yi[1];
    uint4 xrl[1], xil[1], yrl[1], yil[1];
    if constexpr (BF)
        ns_load_chunks<L, 1>(Are, Aim, Bre, Bim, (int64_t)lk + (int64_t)(i0 + lr) * npad,
                             (int64_t)lk + (int64_t)(j0 + lr) * npad, xr, xi, yr, yi);
    if constexpr (X3)
        ns_load_chunks<L, 1>(Are + lo_off, Aim + lo_off, Bre + lo_off, Bim + lo_off,
                             (int64_t)lk + (int64_t)(i0 + lr) * npad, (int64_t)lk + (int64_t)(j0 + lr) * npad, xrl,
                             xil, yrl, yil);
    for (int k0 = 0; k0 < npad; k0 += 32) {
        if constexpr (BF) {
            uint4 ai = xi[0];
            ai.x ^= 0x80008000u; ai.y ^= 0x80008000u; ai.z ^= 0x80008000u; ai.w ^= 0x80008000u;  // conj
            *reinterpret_cast<uint4 *>(&sAr[lr][lks]) = xr[0];
            *reinterpret_cast<uint4 *>(&sAi[lr][lks]) = ai;
            *reinterpret_cast<uint4 *>(&sBr[lr][lks]) = yr[0];
            *reinterpret_cast<uint4 *>(&sBi[lr][lks]) = yi[0];
            if constexpr (X3) {
                uint4 al = xil[0];
                al.x ^= 0x80008000u; al.y ^= 0x80008000u; al.z ^= 0x80008000u; al.w ^= 0x80008000u;
                *reinterpret_cast<uint4 *>(&sArl[lr][lks]) = xrl[0];
                *reinterpret_cast<uint4 *>(&sAil[lr][lks]) = al;
                *reinterpret_cast<uint4 *>(&sBrl[lr][lks]) = yrl[0];
                *reinterpret_cast<uint4 *>(&sBil[lr][lks]) = yil[0];
            }
        } else {
            const int64_t ao = (int64_t)(k0 + lk) + (int64_t)(i0 + lr) * npad;
            const int64_t bo = (int64_t)(k0 + lk) + (int64_t)(j0 + lr) * npad;
#pragma unroll
            for (int h = 0; h < 8; h += 4) {
                const float4 ar = *reinterpret_cast<const float4 *>(Are + ao + h);
                const float4 ai = *reinterpret_cast<const float4 *>(Aim + ao + h);
                *reinterpret_cast<float4 *>(&sAr[lr][lk + h]) = ar;
                *reinterpret_cast<float4 *>(&sAi[lr][lk + h]) = make_float4(-ai.x, -ai.y, -ai.z, -ai.w);
                *reinterpret_cast<float4 *>(&sBr[lr][lk + h]) = *reinterpret_cast<const float4 *>(Bre + bo + h);
                *reinterpret_cast<float4 *>(&sBi[lr][lk + h]) = *reinterpret_cast<const float4 *>(Bim + bo + h);
            }
        }
        __syncthreads();
        if constexpr (BF) {
            const int kn = k0 + 32 < npad ? k0 + 32 : k0;  // the last slice again at the end: no branch
            ns_load_chunks<L, 1>(Are, Aim, Bre, Bim, (int64_t)(kn + lk) + (int64_t)(i0 + lr) * npad,
                                 (int64_t)(kn + lk) + (int64_t)(j0 + lr) * npad, xr, xi, yr, yi);
            if constexpr (X3)
                ns_load_chunks<L, 1>(Are + lo_off, Aim + lo_off, Bre + lo_off, Bim + lo_off,
                                     (int64_t)(kn + lk) + (int64_t)(i0 + lr) * npad,
                                     (int64_t)(kn + lk) + (int64_t)(j0 + lr) * npad, xrl, xil, yrl, yil);
        }
        const int ii = lane & 15, kg = lane >> 4;
        if constexpr (BF) {
            // 32x32x16 operands: row lane % 32 of the wave's 32 rows, k chunk
            // 2h + lane / 32 (rows 32 apart share the swizzle)
            const int rl = lane & 31, kh = lane >> 5;
            const int fsw = ((rl >> 2) ^ (rl >> 1)) & 3;
            if (!idle) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int pos = ((2 * h + kh) ^ fsw) * 8;
                    const v8bf ar = *reinterpret_cast<const v8bf *>(&sAr[wm * 32 + rl][pos]);
                    uint4 u = *reinterpret_cast<const uint4 *>(&sAi[wm * 32 + rl][pos]);  // -Im of the stored column
                    const v8bf ai = *reinterpret_cast<const v8bf *>(&u);
                    u.x ^= 0x80008000u; u.y ^= 0x80008000u; u.z ^= 0x80008000u; u.w ^= 0x80008000u;
                    const v8bf ain = *reinterpret_cast<const v8bf *>(&u);
                    const v8bf br = *reinterpret_cast<const v8bf *>(&sBr[wn * 32 + rl][pos]);
                    const v8bf bi = *reinterpret_cast<const v8bf *>(&sBi[wn * 32 + rl][pos]);
                    if constexpr (X3) {
                        // the cross terms first (the small ones), then hi * hi
                        const v8bf arl = *reinterpret_cast<const v8bf *>(&sArl[wm * 32 + rl][pos]);
                        uint4 ul = *reinterpret_cast<const uint4 *>(&sAil[wm * 32 + rl][pos]);
                        const v8bf ail = *reinterpret_cast<const v8bf *>(&ul);
                        ul.x ^= 0x80008000u; ul.y ^= 0x80008000u; ul.z ^= 0x80008000u; ul.w ^= 0x80008000u;
                        const v8bf ainl = *reinterpret_cast<const v8bf *>(&ul);
                        const v8bf brl = *reinterpret_cast<const v8bf *>(&sBrl[wn * 32 + rl][pos]);
                        const v8bf bil = *reinterpret_cast<const v8bf *>(&sBil[wn * 32 + rl][pos]);
                        accr32 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar, brl, accr32, 0, 0, 0);
                        accr32 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl, br, accr32, 0, 0, 0);
                        acci32 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar, bil, acci32, 0, 0, 0);
                        acci32 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl, bi, acci32, 0, 0, 0);
                        accr32 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ain, bil, accr32, 0, 0, 0);
                        accr32 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ainl, bi, accr32, 0, 0, 0);
                        acci32 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ai, brl, acci32, 0, 0, 0);
                        acci32 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ail, br, acci32, 0, 0, 0);
                    }
                    accr32 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar, br, accr32, 0, 0, 0);
                    acci32 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar, bi, acci32, 0, 0, 0);
                    accr32 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ain, bi, accr32, 0, 0, 0);
                    acci32 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ai, br, acci32, 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < 32; ks += 4) {
                float ar[2], ai[2], br[2], bi[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    ar[a] = sAr[wm * 32 + a * 16 + ii][ks + kg];
                    ai[a] = sAi[wm * 32 + a * 16 + ii][ks + kg];
                }
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    br[b] = sBr[wn * 32 + b * 16 + ii][ks + kg];
                    bi[b] = sBi[wn * 32 + b * 16 + ii][ks + kg];
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[a], br[b], accr[a][b], 0, 0, 0);
                        accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[a], bi[b], accr[a][b], 0, 0, 0);
                        acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[a], bi[b], acci[a][b], 0, 0, 0);
                        acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[a], br[b], acci[a][b], 0, 0, 0);
                    }
            }
        }
        __syncthreads();
    }
    if constexpr (BF) {
        if (!idle)
            ns_store_block32<SPLIT>(accr32, acci32, i0 + wm * 32, j0 + wn * 32, lane, npad, epi, c, Cre, Cim, C64,
                                    ld64, n, lo_off);
        return;
    }
    // epilogue; f32-accumulating 16x16 MFMA layout: D[i][j] in lane
    // j + 16*(i/4), element i % 4
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + wm * 32 + a * 16 + 4 * (lane >> 4) + v;
                const int j = j0 + wn * 32 + b * 16 + (lane & 15);
                if (i < j) continue;  // the mirror of (j, i) covers it
                float re = accr[a][b][v], im = acci[a][b][v];
                if (epi == NS_EPI_T) { re = (i == j ? 3.0f : 0.0f) - c * re; im = -c * im; }
                else { re *= c; im *= c; }
                if (i == j) im = 0.0f;
                if (epi != NS_EPI_F64) {
                    const L lr = to_low<L>(re), li = to_low<L>(im), lni = to_low<L>(-im);
                    const int64_t o = (int64_t)i + (int64_t)j * npad, om = (int64_t)j + (int64_t)i * npad;
                    Cre[o] = lr; Cim[o] = li;
                    Cre[om] = lr; Cim[om] = lni;
                } else if (i < n && j < n) {
                    C64[i + (int64_t)j * ld64] = cmk((double)re, (double)im);
                    C64[j + (int64_t)i * ld64] = cmk((double)re, -(double)im);
                }
            }
}

// ---- BF16 product of the large blocks: 128x128 tiles fed by direct
// global->LDS loads.
//
// The 64x64 tile above stages its operands through registers; at large n its
// MFMAs wait on the loads of the next k-slice.  Here each wave streams one
// operand plane (Re A, Im A, Re B, Im B) straight into LDS with
// global_load_lds_dwordx4 (no registers, no LDS store instructions), into a
// two-deep ring: slice s + 1 is in flight while slice s feeds the MFMAs.
// 4 waves in 2x2 own 64x64 each (4x4 blocks of 16x16x32 MFMA); LDS rows are
// 64 bytes unpadded, the 16-byte chunk q of row r at position q ^ f(r),
// f(r) = ((r >> 2) ^ (r >> 1)) & 3, which keeps every fragment read free of
// bank conflicts (16 lanes over 64 banks or 8 lanes over 32).  Two
// workgroups fit on a CU (64 KiB of LDS, at most 256 registers each).
//
// Tile count: the lower tiles of an npad x npad product, T = m (m + 1) / 2
// with m = npad / 128 rounded up.  When T slightly exceeds the resident
// workgroups (NS_SLOTS), the last T mod NS_SLOTS tiles would run alone in a
// second round; instead each is split along k into `split` parts written
// as raw FP32 partials, summed in part order (deterministic) by a second
// kernel that applies the same epilogue.
constexpr int NS_SLOTS = 512;  // 256 CUs x 2 resident workgroups
constexpr int NS_BIG = NS_BIG_DEFAULT;  // npad from which the 128x128 path is used by default
constexpr int NS_PART_FLOATS = 32768;  // raw accumulators of one tile part

// Tail split of the 128x128 path for an npad x npad product (per block:
// independent of the group size, so group members match single calls).
// slots: resident workgroups of the kernel (NS_SLOTS for BF16; half for the
// split-BF16 form, whose doubled LDS ring leaves one workgroup per CU).
void ns_tail_plan(int npad, int *ntile, int *tfull, int *rem, int *split, int slots = NS_SLOTS) {
    const int m = (npad + 127) / 128, T = m * (m + 1) / 2;
    int r = T > slots ? T % slots : 0;
    if (r > slots / 4) r = 0;
    *ntile = T;
    *rem = r;
    *split = r ? std::min(16, slots / r) : 1;
    *tfull = T - r;
}

// One 16-byte chunk per lane from g into LDS at lds + 16 * lane.  Issued as
// inline assembly so that the compiler does not hold every LDS read behind
// it (it cannot tell the ring slots apart); the waits are explicit: WAIT_VM
// on this wave's own loads, then a barrier for everyone's.
__device__ __forceinline__ void dma16(const void *g, unsigned lds) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(g), "s"(lds) : "memory", "m0");
}
#define NS_WAIT_VM0() __builtin_amdgcn_s_waitcnt((0x7 << 4) | (0xF << 8))

__device__ __forceinline__ void ns_tile_ij(int tb, int &ti, int &tj) {
    ti = (int)((sqrt(8.0 * tb + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= tb) ++ti;
    while (ti * (ti + 1) / 2 > tb) --ti;
    tj = tb - ti * (ti + 1) / 2;
}

// Tile number o of the m x m lower tile triangle in blocked order: squares
// of NS_SUPER x NS_SUPER tiles (J <= I, row by row), each row by row inside
// (the diagonal squares over their lower triangle).  Consecutive numbers
// share few row and column panels, so the contiguous run of tiles that one
// XCD takes (xcd_tile) reuses its operand panels from that XCD's L2.
constexpr int NS_SUPER = 8;
__device__ __forceinline__ void ns128_tile(int o, int m, int &ti, int &tj) {
    const int M = (m + NS_SUPER - 1) / NS_SUPER;
    for (int I = 0; I < M; ++I) {
        const int r = min(NS_SUPER, m - I * NS_SUPER);
        for (int J = 0; J <= I; ++J) {
            const int c = min(NS_SUPER, m - J * NS_SUPER);
            const int cnt = I == J ? r * (r + 1) / 2 : r * c;
            if (o < cnt) {
                int li, lj;
                if (I == J) ns_tile_ij(o, li, lj);
                else { li = o / c; lj = o - li * c; }
                ti = I * NS_SUPER + li;
                tj = J * NS_SUPER + lj;
                return;
            }
            o -= cnt;
        }
    }
    ti = tj = 0;  // not reached for o < m (m + 1) / 2
}

// Epilogue of one 16x16 block at (ib, jb) as in ns_gemm_kernel: the lower
// part with its conjugate mirror; blocks strictly below the diagonal write
// four consecutive rows per lane as one 8-byte store.
template <int SPLIT = 1>
__device__ __forceinline__ void ns128_store_block(const v4f &accr, const v4f &acci, int ib, int jb, int lane, int npad,
                                                  int epi, float c, __bf16 *Cre, __bf16 *Cim, double2 *C64,
                                                  int64_t ld64, int n, int64_t lo_off = 0) {
    if (ib < jb || ib >= npad) return;
    const int ir = ib + 4 * (lane >> 4), j = jb + (lane & 15);
    if (epi != NS_EPI_F64 && ib > jb) {
        union { __bf16 h[4]; uint2 u; } pr, pi, pn, qr, qi, qn;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float re = accr[v], im = acci[v];
            if (epi == NS_EPI_T) { re = -c * re; im = -c * im; }
            else { re *= c; im *= c; }
            if constexpr (SPLIT == 2) {
                bf16_split(re, pr.h[v], qr.h[v]);
                bf16_split(im, pi.h[v], qi.h[v]);
                pn.h[v] = -pi.h[v];
                qn.h[v] = -qi.h[v];
            } else {
                pr.h[v] = (__bf16)re;
                pi.h[v] = (__bf16)im;
                pn.h[v] = (__bf16)(-im);
            }
        }
        const int64_t o = (int64_t)ir + (int64_t)j * npad;
        *reinterpret_cast<uint2 *>(Cre + o) = pr.u;
        *reinterpret_cast<uint2 *>(Cim + o) = pi.u;
        if constexpr (SPLIT == 2) {
            *reinterpret_cast<uint2 *>(Cre + lo_off + o) = qr.u;
            *reinterpret_cast<uint2 *>(Cim + lo_off + o) = qi.u;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t om = (int64_t)j + (int64_t)(ir + v) * npad;
            Cre[om] = pr.h[v];
            Cim[om] = pn.h[v];
            if constexpr (SPLIT == 2) {
                Cre[lo_off + om] = qr.h[v];
                Cim[lo_off + om] = qn.h[v];
            }
        }
        return;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = ir + v;
        if (i < j) continue;
        float re = accr[v], im = acci[v];
        if (epi == NS_EPI_T) { re = (i == j ? 3.0f : 0.0f) - c * re; im = -c * im; }
        else { re *= c; im *= c; }
        if (i == j) im = 0.0f;
        if (epi != NS_EPI_F64) {
            const int64_t o = (int64_t)i + (int64_t)j * npad, om = (int64_t)j + (int64_t)i * npad;
            if constexpr (SPLIT == 2) {
                __bf16 hr, lr, hi, li;
                bf16_split(re, hr, lr);
                bf16_split(im, hi, li);
                Cre[o] = hr; Cim[o] = hi;
                Cre[om] = hr; Cim[om] = -hi;
                Cre[lo_off + o] = lr; Cim[lo_off + o] = li;
                Cre[lo_off + om] = lr; Cim[lo_off + om] = -li;
            } else {
                const __bf16 lr = (__bf16)re, li = (__bf16)im, lni = (__bf16)(-im);
                Cre[o] = lr; Cim[o] = li;
                Cre[om] = lr; Cim[om] = lni;
            }
        } else if (i < n && j < n) {
            C64[i + (int64_t)j * ld64] = cmk((double)re, (double)im);
            C64[j + (int64_t)i * ld64] = cmk((double)re, -(double)im);
        }
    }
}

// Workgroups g < tfull: whole tiles (XCD-aware order); the rest: part
// (g - tfull) % split of tail tile tfull + (g - tfull) / split.
// SPLIT = 2: the split-BF16 products (see ns_gemm_kernel): every wave also
// streams the lo plane of its operand plane (lo_off elements on) into a
// second half of the ring, and each real product takes three MFMAs; the
// ring doubles to 128 KiB, one workgroup per CU.
template <int SPLIT>
__global__ void __launch_bounds__(256, 3 - SPLIT) ns_gemm128_kernel(const __bf16 *Are, const __bf16 *Aim,
                                                                   const __bf16 *Bre, const __bf16 *Bim, int npad,
                                                                   int epi, float c, __bf16 *Cre, __bf16 *Cim,
                                                                   double2 *C64, int64_t ld64, int n, int tfull,
                                                                   int split, float *part, int64_t zs,
                                                                   int64_t lo_off) {
    constexpr bool X3 = SPLIT == 2;
    {
        const int mb = blockIdx.z;
        Are = member_ptr(Are, zs, mb);
        Aim = member_ptr(Aim, zs, mb);
        Bre = member_ptr(Bre, zs, mb);
        Bim = member_ptr(Bim, zs, mb);
        Cre = member_ptr(Cre, zs, mb);
        Cim = member_ptr(Cim, zs, mb);
        C64 = member_ptr(C64, zs, mb);
        part = member_ptr(part, zs, mb);
    }
    // [slot][plane: Re A, Im A, Re B, Im B (then their lo terms)][128 rows x 64 bytes, swizzled]
    __shared__ __align__(16) char lds[2][4 * SPLIT][8192];
    const int g = blockIdx.x;
    const int q = g < tfull ? -1 : g - tfull;
    const int tb = q < 0 ? xcd_tile(g, tfull) : tfull + q / split;
    int ti, tj;
    ns128_tile(tb, (npad + 127) / 128, ti, tj);
    const int i0 = ti * 128, j0 = tj * 128;
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6), wm = w & 1, wn = w >> 1;
    const bool idle = ti == tj && wm == 0 && wn == 1;  // wave tile above the diagonal
    v4f accr[4][4], acci[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) { accr[a][b] = v4f{0, 0, 0, 0}; acci[a][b] = v4f{0, 0, 0, 0}; }
    // wave w streams plane w: lane l fills slot 64 p + l of the plane (row
    // 16 p + l / 4, position l % 4) with the chunk that the swizzle puts
    // there.  Rows past npad (the last tile row when npad % 128 == 64) read
    // row npad - 1 instead: they only feed outputs that are not stored.
    const __bf16 *src = w == 0 ? Are : w == 1 ? Aim : w == 2 ? Bre : Bim;
    const int r0 = w < 2 ? i0 : j0;
    const int cg = (lane & 3) ^ (((lane >> 4) ^ (lane >> 3)) & 3);
    int64_t goff[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) goff[p] = (int64_t)min(r0 + p * 16 + (lane >> 2), npad - 1) * npad + cg * 8;
    const int nkall = npad / 32;
    int kbeg = 0, kend = nkall;
    if (q >= 0) {
        const int kc = (nkall + split - 1) / split;
        kbeg = min(nkall, (q % split) * kc);
        kend = min(nkall, kbeg + kc);
    }
    const unsigned lds0 = (unsigned)(size_t)(__attribute__((address_space(3))) char *)&lds[0][w][0];
#define NS128_ISSUE(ST)                                                          \
    {                                                                            \
        const unsigned dst = lds0 + (unsigned)((ST) & 1) * (4 * SPLIT * 8192);   \
        const __bf16 *s0 = src + (ST) * 32;                                      \
        _Pragma("unroll") for (int p = 0; p < 8; ++p) dma16(s0 + goff[p], dst + p * 1024); \
        if constexpr (X3) {                                                      \
            _Pragma("unroll") for (int p = 0; p < 8; ++p)                        \
                dma16(s0 + lo_off + goff[p], dst + 4 * 8192 + p * 1024);         \
        }                                                                        \
    }
    if (kbeg < kend) NS128_ISSUE(kbeg)
    const int ii = lane & 15, kg = lane >> 4;
    const int rsw = (kg ^ (((ii >> 2) ^ (ii >> 1)) & 3)) * 16;
    for (int s = kbeg; s < kend; ++s) {
        NS_WAIT_VM0();
        asm volatile("s_barrier" ::: "memory");
        if (s + 1 < kend) NS128_ISSUE(s + 1)
        if (!idle) {
            const char *bA = &lds[s & 1][0][0];
            v8bf br[4], bi[4], brl[4], bil[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int off = (wn * 64 + b * 16 + ii) * 64 + rsw;
                br[b] = *reinterpret_cast<const v8bf *>(bA + 2 * 8192 + off);
                bi[b] = *reinterpret_cast<const v8bf *>(bA + 3 * 8192 + off);
                if constexpr (X3) {
                    brl[b] = *reinterpret_cast<const v8bf *>(bA + 6 * 8192 + off);
                    bil[b] = *reinterpret_cast<const v8bf *>(bA + 7 * 8192 + off);
                }
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int off = (wm * 64 + a * 16 + ii) * 64 + rsw;
                const v8bf ar = *reinterpret_cast<const v8bf *>(bA + off);
                // Im of the stored column is -Im A(i, k) (A(i,k) = conj of the
                // stored (k, i)): ai enters Re C with +, its negation Im C
                uint4 u = *reinterpret_cast<const uint4 *>(bA + 8192 + off);
                const v8bf ai = *reinterpret_cast<const v8bf *>(&u);
                u.x ^= 0x80008000u; u.y ^= 0x80008000u; u.z ^= 0x80008000u; u.w ^= 0x80008000u;
                const v8bf ain = *reinterpret_cast<const v8bf *>(&u);
                if constexpr (X3) {
                    // lo terms of the A fragment, then the cross terms (the small ones first)
                    const v8bf arl = *reinterpret_cast<const v8bf *>(bA + 4 * 8192 + off);
                    uint4 ul = *reinterpret_cast<const uint4 *>(bA + 5 * 8192 + off);
                    const v8bf ail = *reinterpret_cast<const v8bf *>(&ul);
                    ul.x ^= 0x80008000u; ul.y ^= 0x80008000u; ul.z ^= 0x80008000u; ul.w ^= 0x80008000u;
                    const v8bf ainl = *reinterpret_cast<const v8bf *>(&ul);
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, brl[b], accr[a][b], 0, 0, 0);
                        accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl, br[b], accr[a][b], 0, 0, 0);
                        accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, bil[b], accr[a][b], 0, 0, 0);
                        accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ail, bi[b], accr[a][b], 0, 0, 0);
                        acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, bil[b], acci[a][b], 0, 0, 0);
                        acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl, bi[b], acci[a][b], 0, 0, 0);
                        acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ain, brl[b], acci[a][b], 0, 0, 0);
                        acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ainl, br[b], acci[a][b], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, br[b], accr[a][b], 0, 0, 0);
                    accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, bi[b], accr[a][b], 0, 0, 0);
                    acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, bi[b], acci[a][b], 0, 0, 0);
                    acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ain, br[b], acci[a][b], 0, 0, 0);
                }
            }
        }
    }
#undef NS128_ISSUE
    if (idle) return;
    if (q >= 0) {
        // raw partial sums: per (wave, block) 64 lanes x 4 values, one
        // 16-byte store per lane and plane
        float *pp = part + (int64_t)q * NS_PART_FLOATS;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int idx = ((w * 16 + a * 4 + b) * 64 + lane) * 4;
                *reinterpret_cast<v4f *>(pp + idx) = accr[a][b];
                *reinterpret_cast<v4f *>(pp + NS_PART_FLOATS / 2 + idx) = acci[a][b];
            }
        return;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            ns128_store_block<SPLIT>(accr[a][b], acci[a][b], i0 + wm * 64 + a * 16, j0 + wn * 64 + b * 16, lane,
                                     npad, epi, c, Cre, Cim, C64, ld64, n, lo_off);
}

// Tail tile tfull + blockIdx.x: its split partials summed in part order,
// then the epilogue; workgroup y covers the 16x16 block (a, b) = (y / 4,
// y % 4) of every wave.
template <int SPLIT>
__global__ void __launch_bounds__(256) ns128_tail_kernel(const float *__restrict__ part, int tfull, int split, int npad,
                                                         int epi, float c, __bf16 *Cre, __bf16 *Cim, double2 *C64,
                                                         int64_t ld64, int n, int64_t zs, int64_t lo_off) {
    {
        const int mb = blockIdx.z;
        part = member_ptr(part, zs, mb);
        Cre = member_ptr(Cre, zs, mb);
        Cim = member_ptr(Cim, zs, mb);
        C64 = member_ptr(C64, zs, mb);
    }
    const int a = blockIdx.y >> 2, b = blockIdx.y & 3;
    int ti, tj;
    ns128_tile(tfull + (int)blockIdx.x, (npad + 127) / 128, ti, tj);
    const int i0 = ti * 128, j0 = tj * 128;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w & 1, wn = w >> 1;
    if (ti == tj && wm == 0 && wn == 1) return;
    const float *pp = part + (int64_t)blockIdx.x * split * NS_PART_FLOATS + ((w * 16 + a * 4 + b) * 64 + lane) * 4;
    v4f re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
    for (int p = 0; p < split; ++p) {
        re += *reinterpret_cast<const v4f *>(pp + (int64_t)p * NS_PART_FLOATS);
        im += *reinterpret_cast<const v4f *>(pp + (int64_t)p * NS_PART_FLOATS + NS_PART_FLOATS / 2);
    }
    ns128_store_block<SPLIT>(re, im, i0 + wm * 64 + a * 16, j0 + wn * 64 + b * 16, lane, npad, epi, c, Cre, Cim, C64,
                             ld64, n, lo_off);
}

// Assembly of Pi = X/2 + (X S + S X)/4 from F = X S (full FP64 product):
// (S X)_ij = conj(F_ji), since X and S are Hermitian, so each lower entry
// needs F_ij and F_ji.  The Hermitian part is what the exact sign would give
// (X and sign X commute); the anti-Hermitian part C = F - F^H = [X, S] is the
// commutator, zero for the exact sign: its norm measures how far S's
// eigenvectors are from X's.  One workgroup per 32x32 lower tile (I >= J)
// loads tile (I, J) and, through LDS, tile (J, I); it writes the svec and
// five partial sums: ||C||_F^2, ||Pi||_F^2, tr S, ||X||_F^2, ||F||_F^2.
constexpr int AT = 32;
constexpr int ASM_SUMS = 5;
__global__ void __launch_bounds__(256) mx_assemble_kernel(const double2 *__restrict__ M,
                                                          const double2 *__restrict__ F,
                                                          const double2 *__restrict__ S, int64_t lda, int n,
                                                          double *y, const int64_t *__restrict__ ioff,
                                                          const int *status, double *red_out, int64_t zs) {
    __shared__ double2 U[AT][AT + 1];
    __shared__ double red[8];
    const int mb = blockIdx.z;
    M = member_ptr(M, zs, mb);
    F = member_ptr(F, zs, mb);
    S = member_ptr(S, zs, mb);
    status = member_ptr(status, zs, mb);
    red_out = member_ptr(red_out, zs, mb);
    if (ioff) y += ioff[mb];
    const int tile = blockIdx.x;
    int I = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= tile) ++I;
    while (I * (I + 1) / 2 > tile) --I;
    const int J = tile - I * (I + 1) / 2;
    const int i0 = I * AT, j0 = J * AT, t = threadIdx.x;
    // tile (J, I) of F: U[ii][jj] = F(j0 + jj, i0 + ii)
#pragma unroll
    for (int q = 0; q < AT * AT / 256; ++q) {
        const int jj = t % AT, ii = t / AT + q * (256 / AT);
        const int r = j0 + jj, c = i0 + ii;
        U[ii][jj] = (r < n && c < n) ? F[r + (int64_t)c * lda] : cmk(0.0, 0.0);
    }
    __syncthreads();
    const bool poison = status[2] == ST_ENONFINITE;
    const double rt2 = 1.41421356237309504880, nan = __builtin_nan("");
    double c2 = 0.0, p2 = 0.0, trs = 0.0, x2 = 0.0, f2 = 0.0;
#pragma unroll
    for (int q = 0; q < AT * AT / 256; ++q) {
        const int ii = t % AT, jj = t / AT + q * (256 / AT);
        const int i = i0 + ii, j = j0 + jj;
        if (i >= n || j >= n || i < j) continue;
        const double2 fij = F[i + (int64_t)j * lda], fji = U[ii][jj], m = M[i + (int64_t)j * lda];
        const double2 h = cmk(0.25 * (fij.x + fji.x), 0.25 * (fij.y - fji.y));
        const double2 out = cmk(0.5 * m.x + h.x, 0.5 * m.y + h.y);
        const double2 cm = cmk(fij.x - fji.x, fij.y + fji.y);
        if (i == j) {
            const double o = 0.5 * m.x + 0.5 * fij.x;
            y[svec_col_start(n, j)] = poison ? nan : o;
            c2 += cabs2(cm);
            p2 += o * o;
            x2 += m.x * m.x;
            f2 += cabs2(fij);
            trs += S[i + (int64_t)i * lda].x;
        } else {
            const int64_t o = svec_off(n, i, j);
            y[o] = poison ? nan : rt2 * out.x;
            y[o + 1] = poison ? nan : rt2 * out.y;
            c2 += 2.0 * cabs2(cm);
            p2 += 2.0 * cabs2(out);
            x2 += 2.0 * cabs2(m);
            f2 += cabs2(fij) + cabs2(fji);
        }
    }
    c2 = block_sum(c2, red);
    p2 = block_sum(p2, red);
    trs = block_sum(trs, red);
    x2 = block_sum(x2, red);
    f2 = block_sum(f2, red);
    if (t == 0) {
        double *o = red_out + (int64_t)tile * ASM_SUMS;
        o[0] = c2; o[1] = p2; o[2] = trs; o[3] = x2; o[4] = f2;
    }
}

// Info record of a mixed projection: the tile partials summed in tile order
// (deterministic), n_pos = (n + tr S) / 2, and a first-order estimate of the
// relative error from its two parts (relative to ||X||_F when Pi = 0):
//  * eigenvectors: in the eigenbasis of X the error of the assembled Pi on an
//    entry coupling eigenvalues of opposite signs is
//    (l_i + l_j) / (l_i - l_j) C_ij / 4, of modulus at most |C_ij| / 4:
//    ||C||_F / 4;
//  * eigenvalues: S's eigenvalue s_i in place of sgn l_i costs
//    |l_i| (1 - |s_i|) / 2 <= |l_i| (1 - s_i^2) / 4 (the iterations keep
//    |s_i| <= 1), and sum l_i^2 (1 - s_i^2) = ||X||_F^2 - ||X S||_F^2, so
//    their share is at most sqrt(||X||_F^2 - ||F||_F^2) / 4.
// The two parts add in quadrature (different entries of the eigenbasis).
__global__ void __launch_bounds__(256) mx_info_kernel(const double *__restrict__ red_in, int ntile, int n, int iters,
                                                      const double *alpha, const int *status, psd_dev_info *info,
                                                      int64_t zs, const int *infoidx) {
    __shared__ double red[8];
    red_in = member_ptr(red_in, zs, blockIdx.z);
    alpha = member_ptr(alpha, zs, blockIdx.z);
    status = member_ptr(status, zs, blockIdx.z);
    if (info) info += infoidx ? infoidx[blockIdx.z] : blockIdx.z;
    double acc[ASM_SUMS] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < ntile; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < ASM_SUMS; ++k) acc[k] += red_in[(int64_t)b * ASM_SUMS + k];
#pragma unroll
    for (int k = 0; k < ASM_SUMS; ++k) acc[k] = block_sum(acc[k], red);
    if (threadIdx.x == 0 && info) {
        const double en = sqrt(acc[0] + fmax(acc[3] - acc[4], 0.0)), pn = sqrt(acc[1]), xn = sqrt(acc[3]);
        const int npos = (int)llround(0.5 * (n + acc[2]));
        info->status = status[2];
        info->n_pos = min(max(npos, 0), n);
        info->n_neg = n - info->n_pos;
        info->iters = iters;
        info->fallback = 0;
        info->reserved = 0;
        info->est_rel_err = pn > 0.0 ? 0.25 * en / pn : (xn > 0.0 ? 0.25 * en / xn : 0.0);
        info->scale = *alpha;
    }
}

// Scalings a_k of the scaled Newton-Schulz steps X <- (a/2) X (3I - a^2 X^2)
// (Chen and Chow, 2014), capped at 1.5.  a_0 = 1 maps a spectrum inside
// (-sqrt 3, sqrt 3) into [-1, 1]; then, with [l, 1] bounding the eigenvalue
// magnitudes, a = min(1.5, sqrt(3 / (1 + l + l^2))) and
// l <- min(f(a l), f(a)), f(t) = (3t - t^3)/2.  The uncapped value would
// give f equal values at both ends, but it pushes the converged top of the
// spectrum far down (f(sqrt 3) = 0), and its regrowth in low precision
// amplifies rounding; the cap keeps the unscaled map's accuracy.  iters = 0:
// as many steps as take l from l0 to within 1e-7 of 1 (21 from 1e-6, against
// 40 unscaled), i.e. eigenvalues down to l0 alpha resolved.
//
// l0 = max(1e-6, u/4) for the unit roundoff u of the iterates' format: the
// rounding of X to that format moves its eigenvalues by about u alpha, so
// the sign of an eigenvalue below that is not determined by the iteration
// anyway, and an unconverged one of magnitude below l0 alpha adds at most
// that much to the error (inside the band the error bounds already allow):
// BF16 (u = 2^-8) takes 12 steps, split BF16 (2^-16) 19, FP32 21.
double ns_l0(int mode) {
    const double u = mode == 1 ? 0x1p-8 : mode == 3 ? 0x1p-16 : 0x1p-24;
    return std::max(1e-6, 0.25 * u);
}

std::vector<double> ns_scalings(int iters, double l0) {
    constexpr double tol = 1e-7, amax = 1.5;
    auto cubic = [](double t) { return 0.5 * (3.0 * t - t * t * t); };
    std::vector<double> a(1, 1.0);
    double l = cubic(l0);
    while (iters > 0 ? (int)a.size() < iters : (1.0 - l > tol && a.size() < 200)) {
        const double s = std::min(amax, std::sqrt(3.0 / (1.0 + l + l * l)));
        a.push_back(s);
        l = std::min(cubic(s * l), cubic(s));
    }
    if (iters > 0) a.resize(iters);
    return a;
}

template <typename L, int SPLIT = 1>
hipError_t ns_run(const MixedWs &w, const double *x, double *y, psd_dev_info *info, int iters_req, int corr,
                  hipStream_t st) {
    const std::vector<double> sc = ns_scalings(iters_req, ns_l0(sizeof(L) == 4 ? 2 : SPLIT == 2 ? 3 : 1));
    const int iters = (int)sc.size();
    const int n = w.n, npad = w.npad;
    const int64_t plane = (int64_t)npad * npad;
    L *X = reinterpret_cast<L *>(w.lo0), *T = reinterpret_cast<L *>(w.lo1), *X2 = reinterpret_cast<L *>(w.lo2);
    const int B = w.nmem;
    const int64_t zs = w.zs;
    dim3 sg((npad + 255) / 256, npad, B);
    // split products: the lo planes follow the two hi planes of each matrix
    const int64_t lo_off = SPLIT == 2 ? 2 * plane : 0;
    if constexpr (SPLIT == 2)
        hipLaunchKernelGGL(ns_scale_split_kernel, sg, dim3(256), 0, st, w.M, w.lda, n, npad, w.alpha,
                           reinterpret_cast<__bf16 *>(X), plane, lo_off, zs);
    else
        hipLaunchKernelGGL((ns_scale_kernel<L>), sg, dim3(256), 0, st, w.M, w.lda, n, npad, w.alpha, X, X + plane,
                           zs);
    // BF16 at npad >= w.ns_big: 128x128 tiles with a split tail; otherwise
    // the 64x64 tile (the choice depends on npad and the threshold only, so
    // that group members match single-block calls bit for bit under the
    // same threshold)
    const bool big = sizeof(L) == 2 && npad >= w.ns_big;
    int ntile, tfull, rem, split;
    if (big) ns_tail_plan(npad, &ntile, &tfull, &rem, &split, NS_SLOTS / SPLIT);
    else { const int mt = npad / 64; ntile = mt * (mt + 1) / 2; tfull = ntile; rem = 0; split = 1; }
    // algorithmic count: the n (n + 1) / 2 lower entries of an order-n
    // Hermitian product, n complex multiply-adds (8 flops) each
    const double ns_flops = 8.0 * (double)n * (double)n * (double)(n + 1) / 2.0 * B;
    auto product = [&](const L *A, const L *Bm, int epi, float cf, L *C, double2 *C64) {
        const int slot = timing_begin(KF_NS, st);
        if constexpr (sizeof(L) == 2) {
            if (big) {
                hipLaunchKernelGGL(ns_gemm128_kernel<SPLIT>, dim3(tfull + rem * split, 1, B), dim3(256), 0, st, A,
                                   A + plane, Bm, Bm + plane, npad, epi, cf, C, C + plane, C64, w.lda, n, tfull, split,
                                   w.part, zs, lo_off);
                if (rem)
                    hipLaunchKernelGGL(ns128_tail_kernel<SPLIT>, dim3(rem, 16, B), dim3(256), 0, st, w.part, tfull,
                                       split, npad, epi, cf, C, C + plane, C64, w.lda, n, zs, lo_off);
                timing_end(slot, st, ns_flops);
                return;
            }
        }
        hipLaunchKernelGGL((ns_gemm_kernel<L, SPLIT>), dim3(ntile, 1, B), dim3(256), 0, st, A, A + plane, Bm,
                           Bm + plane, npad, epi, cf, C, C + plane, C64, w.lda, n, zs, lo_off);
        timing_end(slot, st, ns_flops);
    };
    for (int k = 0; k < iters; ++k) {
        product(X, X, (int)NS_EPI_T, (float)(sc[k] * sc[k]), T, (double2 *)nullptr);
        const bool last = k == iters - 1;
        product(X, T, last ? (int)NS_EPI_F64 : (int)NS_EPI_HALF, (float)(0.5 * sc[k]), X2, w.S);
        std::swap(X, X2);
    }
    // FP64 corrections S <- S (3I - S^2) / 2
    double2 *S = w.S, *S2 = w.S2;
    for (int c = 0; c < corr; ++c) {
        GemmDesc a{};
        a.M = a.N = a.K = n;
        a.A = GemmOperand{S, S, w.lda, w.lda, n, OP_N, nullptr};
        a.B = GemmOperand{S, S, w.lda, w.lda, n, OP_N, nullptr};
        a.C = w.T64; a.ldc = w.lda; a.alpha = -1.0; a.beta = 0.0; a.diag_add = 3.0;
        a.lower_only = 1; a.mirror = 1;  // S^2 is Hermitian
        a.nmem = B; a.zs = zs;
        hipError_t e = gemm_launch(a, true, EPI_STORE, st);
        if (e != hipSuccess) return e;
        GemmDesc b{};
        b.M = b.N = b.K = n;
        b.A = GemmOperand{S, S, w.lda, w.lda, n, OP_N, nullptr};
        b.B = GemmOperand{w.T64, w.T64, w.lda, w.lda, n, OP_N, nullptr};
        b.C = S2; b.ldc = w.lda; b.alpha = 0.5; b.beta = 0.0;
        b.lower_only = 1; b.mirror = 1;  // S and 3I - S^2 commute: Hermitian product
        b.nmem = B; b.zs = zs;
        e = gemm_launch(b, true, EPI_STORE, st);
        if (e != hipSuccess) return e;
        std::swap(S, S2);
    }
    // F = X S (full), then the symmetrised assembly and the info record
    GemmDesc f{};
    f.M = f.N = f.K = n;
    f.A = GemmOperand{w.M, w.M, w.lda, w.lda, n, OP_N, nullptr};
    f.B = GemmOperand{S, S, w.lda, w.lda, n, OP_N, nullptr};
    f.C = w.T64; f.ldc = w.lda; f.alpha = 1.0; f.beta = 0.0;
    f.nmem = B; f.zs = zs;
    hipError_t e = gemm_launch(f, true, EPI_STORE, st);
    if (e != hipSuccess) return e;
    const int at = (n + AT - 1) / AT, natile = at * (at + 1) / 2;
    hipLaunchKernelGGL(mx_assemble_kernel, dim3(natile, 1, B), dim3(256), 0, st, w.M, w.T64, S, w.lda, n, y, w.ioff,
                       w.status, w.red, zs);
    hipLaunchKernelGGL(mx_info_kernel, dim3(1, 1, B), dim3(256), 0, st, w.red, natile, n, iters, w.alpha, w.status,
                       info, zs, w.infoidx);
    return hipGetLastError();
}

}  // namespace

size_t mixed_layout(int n, int mode, void *base, MixedWs *w) {
    size_t off = 0;
    char *b = static_cast<char *>(base);
    auto take = [&](size_t bytes) -> void * {
        void *p = b ? b + off : nullptr;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    MixedWs W{};
    W.n = n;
    W.lda = (n + 63) / 64 * 64;
    W.npad = W.lda;
    const size_t lowsz = mode == 1 ? 2 : 4;
    const size_t plane2 = 2 * (size_t)W.npad * W.npad * lowsz;
    const size_t cmat = sizeof(double2) * (size_t)W.lda * n;
    W.M = (double2 *)take(cmat);
    W.S = (double2 *)take(cmat);
    W.S2 = (double2 *)take(cmat);
    W.T64 = (double2 *)take(cmat);
    W.lo0 = take(plane2);
    W.lo1 = take(plane2);
    W.lo2 = take(plane2);
    W.q = (double2 *)take(sizeof(double2) * (size_t)W.lda);
    W.qprev = (double2 *)take(sizeof(double2) * (size_t)W.lda);
    W.wv = (double2 *)take(sizeof(double2) * (size_t)W.lda);
    W.P = (double2 *)take(sizeof(double2) * (size_t)LZ_SPLIT * n);
    W.ab = (double *)take(sizeof(double) * (2 * LZ_STEPS + 8));
    W.alpha = (double *)take(sizeof(double));
    W.status = (int *)take(sizeof(int) * 4);
    {
        const size_t at = ((size_t)n + AT - 1) / AT;
        W.red = (double *)take(sizeof(double) * ASM_SUMS * (at * (at + 1) / 2));
    }
    W.part = nullptr;
    W.ns_big = NS_BIG;
    if ((mode == 1 || mode == 3) && W.npad >= NS_BIG) {
        int ntile, tfull, rem, split;
        ns_tail_plan(W.npad, &ntile, &tfull, &rem, &split, mode == 3 ? NS_SLOTS / 2 : NS_SLOTS);
        if (rem) W.part = (float *)take(sizeof(float) * NS_PART_FLOATS * (size_t)rem * split);
    }
    W.nmem = 1;
    W.zs = 0;
    W.ioff = nullptr;
    W.infoidx = nullptr;
    if (w) *w = W;
    return off;
}

hipError_t mixed_project(const MixedWs &w, int mode, const double *x, double *y, psd_dev_info *info, int iters,
                         int corr, hipStream_t st) {
    const int n = w.n;
    if (iters < 0) iters = 0;
    // automatic corrections: one for BF16, where it tightens the eigenvalue
    // part of the error estimate; none for FP32 and split BF16, whose S is
    // already within their own rounding of S^2 = I (measured: the step
    // changes neither the error nor the estimate there)
    if (corr < 0) corr = mode == 1 ? 1 : 0;
    const int B = w.nmem;
    const int64_t zs = w.zs;
    hipLaunchKernelGGL(mx_init_kernel, dim3(1, 1, B), dim3(64), 0, st, w.status, zs);
    hipLaunchKernelGGL(mx_unpack_kernel, dim3((n + 255) / 256, n, B), dim3(256), 0, st, x, w.M, w.lda, n, w.status, zs,
                       w.ioff);
    // spectral scale
    hipLaunchKernelGGL(lz_init_kernel, dim3(1, 1, B), dim3(1024), 0, st, n, w.q, w.qprev, w.ab, zs);
    const int steps = std::min(LZ_STEPS, n);
    for (int s = 0; s < steps; ++s) {
        hipLaunchKernelGGL(lz_gemv_kernel, dim3((n + 63) / 64, LZ_SPLIT, B), dim3(256), 0, st, w.M, w.lda, n, w.q,
                           w.P, zs);
        hipLaunchKernelGGL(lz_step_kernel, dim3(1, 1, B), dim3(1024), 0, st, n, s, w.P, w.q, w.qprev, w.wv, w.ab, zs);
    }
    hipLaunchKernelGGL(lz_final_kernel, dim3(1, 1, B), dim3(64), 0, st, w.ab, w.alpha, zs);
    if (mode == 1) return ns_run<__bf16>(w, x, y, info, iters, corr, st);
    if (mode == 3) return ns_run<__bf16, 2>(w, x, y, info, iters, corr, st);
    return ns_run<float>(w, x, y, info, iters, corr, st);
}

}  // namespace psd
