// Internal device helpers of the gfx950 PSD-projection library.
//
// Conventions used by every kernel:
//  * A svec block (the paper's vec_R, App. D.1) holds, per row i of the upper
//    triangle of X, X_ii followed by sqrt2 (Re, Im) of X_ij, j > i.  Read as
//    column i of a lower triangle this is the matrix M = X^T = conj(X):
//    M(j,i) = X_ij for j >= i.  Every kernel works on M, column-major.
//    Pi(conj X) = conj Pi(X) and DPi commutes with conjugation, so packing
//    the result with the same rule gives exactly svec(Pi(X)).
//  * Complex values are double2 {re, im}; matrices are column-major with a
//    leading dimension `ld` (elements).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psd {

typedef double2 cd;

__host__ __device__ inline long svec_col_start(int n, int j) { return (long)j * (2L * n - j); }
// Offset of sqrt2*Re M(i,j), i > j (Im follows).
__host__ __device__ inline long svec_off(int n, int i, int j) {
    return svec_col_start(n, j) + 1 + 2L * (i - j - 1);
}

__device__ __forceinline__ cd cmk(double r, double i) { return make_double2(r, i); }
__device__ __forceinline__ cd cadd(cd a, cd b) { return cmk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cd csub(cd a, cd b) { return cmk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cd cmul(cd a, cd b) { return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// conj(a) * b
__device__ __forceinline__ cd cmulc(cd a, cd b) { return cmk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }
__device__ __forceinline__ cd cconj(cd a) { return cmk(a.x, -a.y); }
__device__ __forceinline__ cd cscale(cd a, double s) { return cmk(a.x * s, a.y * s); }
__device__ __forceinline__ double cabs2(cd a) { return a.x * a.x + a.y * a.y; }
// acc + a*b
__device__ __forceinline__ cd cfma(cd a, cd b, cd acc) {
    return cmk(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}
// acc + conj(a)*b
__device__ __forceinline__ cd cfmac(cd a, cd b, cd acc) {
    return cmk(fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.x, b.y, fma(-a.y, b.x, acc.y)));
}
__device__ __forceinline__ cd cdiv(cd a, cd b) {
    // Smith's algorithm
    if (fabs(b.x) >= fabs(b.y)) {
        double r = b.y / b.x, den = b.x + b.y * r;
        return cmk((a.x + a.y * r) / den, (a.y - a.x * r) / den);
    } else {
        double r = b.x / b.y, den = b.x * r + b.y;
        return cmk((a.x * r + a.y) / den, (a.y * r - a.x) / den);
    }
}

__device__ __forceinline__ double warp_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of one double over the 64 lanes of a wave whose lanes are all active,
// the same value in every lane, without LDS traffic: inside each row of 16
// lanes four DPP exchanges (the quad permutations 1,0,3,2 and 2,3,0,1, then
// the half-row and the row mirrors), each pairing a lane with one that holds
// a disjoint partial, so every lane of a row ends with the row's sum (a + b
// and b + a round alike); then the four row sums, read from lanes 0, 16, 32
// and 48, added in that order.
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double readlane_double(double v, int l) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v += dpp_double<0xB1>(v);   // quad_perm(1, 0, 3, 2): lane ^ 1
    v += dpp_double<0x4E>(v);   // quad_perm(2, 3, 0, 1): lane ^ 2
    v += dpp_double<0x141>(v);  // row_half_mirror: lane 7 - i within 8
    v += dpp_double<0x140>(v);  // row_mirror: lane 15 - i within 16
    return ((readlane_double(v, 0) + readlane_double(v, 16)) + readlane_double(v, 32)) + readlane_double(v, 48);
}

// Exchange of a pair of doubles between lane l and lane l ^ O for O = 32
// (the halves of the wave) or O = 16 (even and odd rows of 16 lanes) by the
// lane-swap instructions, without LDS traffic: on return `a` and `b` hold
// the lane's own a and the partner's a where (l & O) == 0, and the
// partner's b and the lane's own b where (l & O) != 0.
template <int O>
__device__ __forceinline__ void lane_swap_pair(double &a, double &b) {
    static_assert(O == 32 || O == 16, "swap distance");
    const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
    const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
    unsigned alo = (unsigned)ua, ahi = (unsigned)(ua >> 32), blo = (unsigned)ub, bhi = (unsigned)(ub >> 32);
    if constexpr (O == 32) {
        const auto lo = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
        alo = lo[0]; blo = lo[1]; ahi = hi[0]; bhi = hi[1];
    } else {
        const auto lo = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
        alo = lo[0]; blo = lo[1]; ahi = hi[0]; bhi = hi[1];
    }
    a = __longlong_as_double((long long)(((unsigned long long)ahi << 32) | alo));
    b = __longlong_as_double((long long)(((unsigned long long)bhi << 32) | blo));
}

// x of lane l ^ O (every lane of the wave active), without LDS traffic:
// lane swaps for 32 and 16; inside a row of 16 lanes DPP: the rotation by 8
// (row_ror:8 is l ^ 8), the shifts by 4 chosen by bit 2 of the lane
// (row_shl:4 reads lane l + 4, row_shr:4 lane l - 4), the quad permutations
// for 2 and 1.
template <int O>
__device__ __forceinline__ double xor_lane(double x, int lane) {
    static_assert(O == 32 || O == 16 || O == 8 || O == 4 || O == 2 || O == 1, "xor distance");
    if constexpr (O == 32 || O == 16) {
        double a = x, b = x;
        lane_swap_pair<O>(a, b);
        return (lane & O) ? a : b;
    } else if constexpr (O == 8) {
        return dpp_double<0x128>(x);
    } else if constexpr (O == 4) {
        const double from_above = dpp_double<0x104>(x);  // row_shl:4
        const double from_below = dpp_double<0x114>(x);  // row_shr:4
        return (lane & 4) ? from_below : from_above;
    } else if constexpr (O == 2) {
        return dpp_double<0x4E>(x);
    } else {
        return dpp_double<0xB1>(x);
    }
}

// Sums K doubles (K a power of two, 2 <= K <= 32) over the 64 lanes of a
// wave whose lanes are all active.  Each exchange stage sends half of the
// live values to the partner lane l ^ O and keeps the other half, so the K
// sums cost K - 1 + log2(64 / K) exchanges instead of K * 6; the exchanges
// across 32 and 16 lanes are lane swaps of a kept/sent pair, the others DPP
// (none goes through LDS).  Lane l returns the total of value l / (64 / K).
template <int CNT, int O, int K>
__device__ __forceinline__ void wave_split_stage(double (&v)[K], int lane) {
    if constexpr (CNT > 1) {
        const bool up = (lane & O) != 0;
#pragma unroll
        for (int i = 0; i < CNT / 2; ++i) {
            if constexpr (O == 32 || O == 16) {
                // lower lanes keep v[i] and receive the partner's v[i];
                // upper lanes keep v[i + CNT/2] and receive the partner's
                double a = v[i], b = v[i + CNT / 2];
                lane_swap_pair<O>(a, b);
                v[i] = up ? b + a : a + b;
            } else {
                const double send = up ? v[i] : v[i + CNT / 2];
                const double keep = up ? v[i + CNT / 2] : v[i];
                v[i] = keep + xor_lane<O>(send, lane);
            }
        }
        wave_split_stage<CNT / 2, O / 2, K>(v, lane);
    }
}

template <int O>
__device__ __forceinline__ double wave_tail_sum(double r, int lane) {
    if constexpr (O > 0) {
        r += xor_lane<O>(r, lane);
        return wave_tail_sum<O / 2>(r, lane);
    } else {
        return r;
    }
}

template <int K>
__device__ __forceinline__ double wave_sum_split(double (&v)[K]) {
    static_assert(K >= 2 && K <= 32 && (K & (K - 1)) == 0, "K");
    const int lane = threadIdx.x & 63;
    wave_split_stage<K, 32, K>(v, lane);
    return wave_tail_sum<32 / K>(v[0], lane);
}

// Block-wide sum of one double; `red` is LDS scratch of >= blockDim/64 doubles.
// All threads receive the total.  Contains two barriers.
__device__ inline double block_sum(double v, double *red) {
    v = warp_sum(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < nw; ++k) t += red[k];
    return t;
}

// Lockstep groups of same-order blocks: member b owns the workspace slot
// b * zs bytes after member 0's, so every workspace pointer of member b is
// member 0's moved by that much (the member index comes from a grid
// dimension; a single block is the group of one with zs = 0).
template <class T>
__device__ __forceinline__ T *member_ptr(T *p, int64_t zs, int b) {
    return (p && b) ? (T *)((const char *)p + (int64_t)b * zs) : p;
}

// Device-side status codes (mirror psd_status).
enum { ST_OK = 0, ST_ENONFINITE = 4, ST_ENOCONV = 5 };

}  // namespace psd
