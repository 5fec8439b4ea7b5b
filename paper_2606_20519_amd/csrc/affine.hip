// Affine step of the SCS iteration for the bipartite process-matrix SDP
// (App. D.1-D.2): the constraint map and its adjoint
//     A x = -sum_mu x_mu F_mu,      (A^T Z)_mu = -tr[F_mu Z],
// over the allowed traceless multi-indices mu = (alpha_1, beta_1, alpha_2,
// beta_2), F_mu = s_a1 (x) s_b1 (x) s_a2 (x) s_b2 on A_i (x) A_o (x) B_i (x) B_o
// (local dimension d, D = d^2 local basis elements s_alpha: the normalised
// generalised Gell-Mann matrices of App. A, eq. gellmann_basis), and the
// closed form z_x = (a_x - A^T a_y)/2, z_y = a_y + A z_x of the affine
// projection when A^T A = I.
//
// The global basis is never formed (as in the paper's own implementation):
// with y reindexed as a 4-mode tensor T[p_1, p_2, p_3, p_4], p_n = (a_n, b_n)
// the row and column digits of subsystem n, tr[F_mu y] is the product of
// four local transforms, one per mode, each a D x D matrix with at most d
// nonzeros per row (s_alpha has 1, 2 or up to d entries).  Each transform is
// one memory-bound pass over the d^8 complex entries; the allowed
// coefficients are gathered to x (or scattered from it) by a closed-form
// rank, and the svec is unpacked / packed in the first and last passes.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/psdproj.h"
#include "common.h"

namespace psd {

namespace {

struct AffGeo {
    int d, D;
    int64_t n;      // d^4: order of y
    int64_t total;  // d^8 = D^4 tensor entries
};

inline AffGeo aff_geo(int d) {
    AffGeo g;
    g.d = d;
    g.D = d * d;
    g.n = (int64_t)g.D * g.D;
    g.total = g.n * g.n;
    return g;
}

// Off-diagonal pair (j, k), j < k, of index s in lexicographic order, and back.
__device__ __forceinline__ int pair_index(int d, int j, int k) { return j * (2 * d - j - 1) / 2 + (k - j - 1); }
__device__ __forceinline__ void pair_of(int d, int s, int &j, int &k) {
    j = 0;
    while (s >= d - 1 - j) {
        s -= d - 1 - j;
        ++j;
    }
    k = j + 1 + s;
}

// Forward local transform: out[alpha] = sum_p s_alpha[b, a] in[p], p = a d + b.
// Writes the nonzeros of row alpha (at most d) to ps / cs; returns the count.
__device__ __forceinline__ int gm_row(int d, int alpha, int *ps, cd *cs) {
    const int P = d * (d - 1) / 2;
    const double rs2 = 0.70710678118654752440;
    if (alpha == 0) {
        const double c = 1.0 / sqrt((double)d);
        for (int a = 0; a < d; ++a) { ps[a] = a * d + a; cs[a] = cmk(c, 0.0); }
        return d;
    }
    if (alpha < d) {  // diagonal element l = alpha - 1
        const int l = alpha - 1;
        const double c = sqrt(1.0 / ((double)(l + 1) * (double)(l + 2)));
        for (int j = 0; j <= l; ++j) { ps[j] = j * d + j; cs[j] = cmk(c, 0.0); }
        ps[l + 1] = (l + 1) * d + (l + 1);
        cs[l + 1] = cmk(-(double)(l + 1) * c, 0.0);
        return l + 2;
    }
    int j, k;
    if (alpha < d + P) {  // symmetric (|j><k| + |k><j|)/sqrt2
        pair_of(d, alpha - d, j, k);
        ps[0] = k * d + j; cs[0] = cmk(rs2, 0.0);
        ps[1] = j * d + k; cs[1] = cmk(rs2, 0.0);
        return 2;
    }
    // antisymmetric -i(|j><k| - |k><j|)/sqrt2: s[j,k] = -i/sqrt2, s[k,j] = +i/sqrt2;
    // the row takes s[b, a]: (a, b) = (k, j) -> s[j,k], (a, b) = (j, k) -> s[k,j]
    pair_of(d, alpha - d - P, j, k);
    ps[0] = k * d + j; cs[0] = cmk(0.0, -rs2);
    ps[1] = j * d + k; cs[1] = cmk(0.0, rs2);
    return 2;
}

// Adjoint local transform: out[p] = sum_alpha s_alpha[a, b] in[alpha],
// p = a d + b.  Nonzeros of row p (at most d) to as_ / cs; returns the count.
__device__ __forceinline__ int gm_col(int d, int p, int *as_, cd *cs) {
    const int P = d * (d - 1) / 2;
    const double rs2 = 0.70710678118654752440;
    const int a = p / d, b = p - a * d;
    if (a == b) {
        int cnt = 0;
        as_[cnt] = 0;
        cs[cnt++] = cmk(1.0 / sqrt((double)d), 0.0);
        for (int l = max(a - 1, 0); l <= d - 2; ++l) {
            const double c = sqrt(1.0 / ((double)(l + 1) * (double)(l + 2)));
            if (a <= l) { as_[cnt] = 1 + l; cs[cnt++] = cmk(c, 0.0); }
            else if (a == l + 1) { as_[cnt] = 1 + l; cs[cnt++] = cmk(-(double)(l + 1) * c, 0.0); }
        }
        return cnt;
    }
    const int j = min(a, b), k = max(a, b), s = pair_index(d, j, k);
    as_[0] = d + s;
    cs[0] = cmk(rs2, 0.0);
    as_[1] = d + P + s;
    cs[1] = (a == j) ? cmk(0.0, -rs2) : cmk(0.0, rs2);
    return 2;
}

// Sector of one party's (alpha, beta): 0 baseline (0, 0), 1 effect-like
// (alpha >= 1, beta = 0), 2 transformation-like (beta >= 1).
__device__ __forceinline__ int sector_of(int alpha, int beta) { return beta >= 1 ? 2 : (alpha >= 1 ? 1 : 0); }

// Effect-like values q' = alpha' D (alpha' >= 1) below q (party index q = alpha D + beta).
__device__ __forceinline__ int effect_below(int D, int q) { return q > 0 ? min(D - 1, (q - 1) / D) : 0; }

// Rank of an allowed mu = (q1, q2), q = alpha D + beta, in the lexicographic
// order of the allowed traceless multi-indices, or -1 if mu is not allowed.
// Allowed sector pairs: (B,E), (E,B), (E,E), (E,T), (T,E); a first party in
// B or T admits D - 1 second parties (the effect-like ones), one in E all D^2.
__device__ __forceinline__ int64_t mu_rank(int D, int q1, int q2) {
    const int s1 = sector_of(q1 / D, q1 % D), s2 = sector_of(q2 / D, q2 % D);
    const bool ok = (s1 == 1) || (s2 == 1);  // some effect-like party (excludes (B,B), (B,T), (T,B), (T,T))
    if (!ok) return -1;
    const int nb = q1 > 0 ? 1 : 0, ne = effect_below(D, q1), nt = q1 - nb - ne;
    const int prefix = nb * (D - 1) + ne * D * D + nt * (D - 1);   // < d^8 <= 2^24
    const int within = (s1 == 1) ? q2 : effect_below(D, q2);
    return prefix + within;
}

// y (svec, order n = d^4) -> T[p1, p2, p3, p4], p_m = a_m d + b_m.
__global__ void __launch_bounds__(256) aff_unpack_kernel(const double *__restrict__ y, cd *T, int d, int64_t total) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    const int D = d * d, n = D * D;
    int a = 0, b = 0;
    unsigned rem = (unsigned)t;   // d^8 <= 2^24
    int mul = 1;
    for (int m = 3; m >= 0; --m) {
        const int p = (int)(rem % (unsigned)D);
        rem /= (unsigned)D;
        a += (p / d) * mul;
        b += (p % d) * mul;
        mul *= d;
    }
    const double rs2 = 0.70710678118654752440;
    cd v;
    if (a == b) {
        v = cmk(y[svec_col_start(n, a)], 0.0);
    } else if (a < b) {
        const int64_t o = svec_off(n, b, a);  // y_ab, a < b: row a of the upper triangle
        v = cmk(y[o] * rs2, y[o + 1] * rs2);
    } else {
        const int64_t o = svec_off(n, a, b);
        v = cmk(y[o] * rs2, -y[o + 1] * rs2);
    }
    T[t] = v;
}

// One local transform along mode m (0 = most significant) of the D^4 tensor
// (d^8 <= 2^24 entries: 32-bit indices).  Each workgroup first tabulates the
// nonzeros of the D rows of the local transform in LDS.
__global__ void __launch_bounds__(256) aff_mode_kernel(const cd *__restrict__ in, cd *out, int d, int m, int adjoint,
                                                       int total) {
    __shared__ int tab_j[64][8];
    __shared__ cd tab_c[64][8];
    __shared__ int tab_n[64];
    const int D = d * d;
    for (int r = threadIdx.x; r < D; r += 256) {
        int js[8];
        cd cs[8];
        const int c = adjoint ? gm_col(d, r, js, cs) : gm_row(d, r, js, cs);
        tab_n[r] = c;
        for (int q = 0; q < c; ++q) {
            tab_j[r][q] = js[q];
            tab_c[r][q] = cs[q];
        }
    }
    __syncthreads();
    const unsigned t = blockIdx.x * 256u + threadIdx.x;
    if (t >= (unsigned)total) return;
    unsigned inner = 1;
    for (int k = m + 1; k < 4; ++k) inner *= (unsigned)D;
    const unsigned hi = t / inner, lo = t - hi * inner;
    const unsigned idx = hi % (unsigned)D;
    const unsigned base = (hi - idx) * inner + lo;
    const int cnt = tab_n[idx];
    cd acc = cmk(0.0, 0.0);
    for (int q = 0; q < cnt; ++q) acc = cfma(tab_c[idx][q], in[base + (unsigned)tab_j[idx][q] * inner], acc);
    out[t] = acc;
}

// Allowed coefficients of c = tr[F_mu y] to x: x = -Re c (A^T y), or
// x = (a_x + Re c)/2 (the affine step's z_x, with A^T a_y = -c).
__global__ void __launch_bounds__(256) aff_gather_kernel(const cd *__restrict__ c, const double *__restrict__ ax,
                                                         double *x, int d, int64_t total) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    const int D = d * d;
    const unsigned DD = (unsigned)(D * D), tt = (unsigned)t;
    const int64_t r = mu_rank(D, (int)(tt / DD), (int)(tt % DD));
    if (r < 0) return;
    const double v = c[t].x;
    x[r] = ax ? 0.5 * (ax[r] + v) : -v;
}

// c[mu] = coef x[rank(mu)] for allowed mu, 0 elsewhere.
__global__ void __launch_bounds__(256) aff_scatter_kernel(const double *__restrict__ x, cd *c, int d, double coef,
                                                          int64_t total) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    const int D = d * d;
    const unsigned DD = (unsigned)(D * D), tt = (unsigned)t;
    const int64_t r = mu_rank(D, (int)(tt / DD), (int)(tt % DD));
    c[t] = r < 0 ? cmk(0.0, 0.0) : cmk(coef * x[r], 0.0);
}

// T -> y (svec), y = base + T (base nullable): each svec entry once, from
// the tensor entry of (a, b), a <= b.
__global__ void __launch_bounds__(256) aff_pack_kernel(const cd *__restrict__ T, const double *base, double *y, int d,
                                                       int64_t total) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    const int D = d * d, n = D * D;
    int a = 0, b = 0;
    unsigned rem = (unsigned)t;   // d^8 <= 2^24
    int mul = 1;
    for (int m = 3; m >= 0; --m) {
        const int p = (int)(rem % (unsigned)D);
        rem /= (unsigned)D;
        a += (p / d) * mul;
        b += (p % d) * mul;
        mul *= d;
    }
    if (a > b) return;
    const double rt2 = 1.41421356237309504880;
    const cd v = T[t];
    if (a == b) {
        const int64_t o = svec_col_start(n, a);
        y[o] = (base ? base[o] : 0.0) + v.x;
    } else {
        const int64_t o = svec_off(n, b, a);
        y[o] = (base ? base[o] : 0.0) + rt2 * v.x;
        y[o + 1] = (base ? base[o + 1] : 0.0) + rt2 * v.y;
    }
}

hipError_t aff_modes(const AffGeo &g, cd *&cur, cd *&other, int adjoint, hipStream_t st) {
    const int grid = (int)((g.total + 255) / 256);
    for (int m = 0; m < 4; ++m) {
        hipLaunchKernelGGL(aff_mode_kernel, dim3(grid), dim3(256), 0, st, cur, other, g.d, m, adjoint, (int)g.total);
        std::swap(cur, other);
    }
    return hipGetLastError();
}

// x = A^T y, or z_x = (a_x - A^T y)/2 when ax is given.  Leaves the buffers swapped.
hipError_t aff_adjoint(const AffGeo &g, const double *y, const double *ax, double *x, cd *b0, cd *b1, hipStream_t st) {
    const int grid = (int)((g.total + 255) / 256);
    hipLaunchKernelGGL(aff_unpack_kernel, dim3(grid), dim3(256), 0, st, y, b0, g.d, g.total);
    cd *cur = b0, *other = b1;
    hipError_t e = aff_modes(g, cur, other, 0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(aff_gather_kernel, dim3(grid), dim3(256), 0, st, cur, ax, x, g.d, g.total);
    return hipGetLastError();
}

// y = base + A x (base nullable).
hipError_t aff_apply(const AffGeo &g, const double *x, const double *base, double *y, cd *b0, cd *b1, hipStream_t st) {
    const int grid = (int)((g.total + 255) / 256);
    hipLaunchKernelGGL(aff_scatter_kernel, dim3(grid), dim3(256), 0, st, x, b0, g.d, -1.0, g.total);
    cd *cur = b0, *other = b1;
    hipError_t e = aff_modes(g, cur, other, 1, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(aff_pack_kernel, dim3(grid), dim3(256), 0, st, cur, base, y, g.d, g.total);
    return hipGetLastError();
}

bool aff_d_ok(int d) { return d >= 2 && d <= 8; }

bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

psd_status aff_check(int d, size_t ws_bytes, const void *ws) {
    if (!aff_d_ok(d)) return PSD_EINVAL;
    size_t need = 0;
    psd_affine_workspace_size(d, &need);
    if (!ws || ws_bytes < need) return PSD_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % 256) return PSD_EINVAL;
    return PSD_OK;
}

}  // namespace

}  // namespace psd

using namespace psd;

extern "C" {

psd_status psd_affine_dims(int32_t d, int64_t *nx, int64_t *ny) {
    if (!aff_d_ok(d) || !nx || !ny) return PSD_EINVAL;
    const int64_t D = (int64_t)d * d;
    *nx = (D - 1) * (2 * D * D - D + 1);
    *ny = D * D * D * D;
    return PSD_OK;
}

psd_status psd_affine_workspace_size(int32_t d, size_t *bytes) {
    if (!aff_d_ok(d) || !bytes) return PSD_EINVAL;
    const AffGeo g = aff_geo(d);
    const size_t one = ((size_t)g.total * sizeof(cd) + 255) / 256 * 256;
    *bytes = 2 * one;
    return PSD_OK;
}

psd_status psd_constraint_adjoint(int32_t d, const double *y, double *x, void *ws, size_t ws_bytes, void *stream) {
    psd_status st = aff_check(d, ws_bytes, ws);
    if (st != PSD_OK) return st;
    if (!y || !x || !aligned8(y) || !aligned8(x)) return PSD_EINVAL;
    const AffGeo g = aff_geo(d);
    const size_t one = ((size_t)g.total * sizeof(cd) + 255) / 256 * 256;
    cd *b0 = static_cast<cd *>(ws), *b1 = reinterpret_cast<cd *>(static_cast<char *>(ws) + one);
    return aff_adjoint(g, y, nullptr, x, b0, b1, static_cast<hipStream_t>(stream)) == hipSuccess ? PSD_OK
                                                                                             : PSD_EDEVICE;
}

psd_status psd_constraint_apply(int32_t d, const double *x, double *y, void *ws, size_t ws_bytes, void *stream) {
    psd_status st = aff_check(d, ws_bytes, ws);
    if (st != PSD_OK) return st;
    if (!y || !x || !aligned8(y) || !aligned8(x)) return PSD_EINVAL;
    const AffGeo g = aff_geo(d);
    const size_t one = ((size_t)g.total * sizeof(cd) + 255) / 256 * 256;
    cd *b0 = static_cast<cd *>(ws), *b1 = reinterpret_cast<cd *>(static_cast<char *>(ws) + one);
    return aff_apply(g, x, nullptr, y, b0, b1, static_cast<hipStream_t>(stream)) == hipSuccess ? PSD_OK
                                                                                          : PSD_EDEVICE;
}

psd_status psd_affine_step(int32_t d, const double *ax, const double *ay, double *zx, double *zy, void *ws,
                           size_t ws_bytes, void *stream) {
    psd_status st = aff_check(d, ws_bytes, ws);
    if (st != PSD_OK) return st;
    if (!ax || !ay || !zx || !zy) return PSD_EINVAL;
    if (!aligned8(ax) || !aligned8(ay) || !aligned8(zx) || !aligned8(zy)) return PSD_EINVAL;
    const AffGeo g = aff_geo(d);
    int64_t nx = 0, ny = 0;
    psd_affine_dims(d, &nx, &ny);
    // zx may alias ax and zy may alias ay; no other overlap
    auto overlap = [](const void *a, size_t na, const void *b, size_t nb) {
        const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
        return pa < pb + nb && pb < pa + na;
    };
    const size_t bx = sizeof(double) * (size_t)nx, by = sizeof(double) * (size_t)ny;
    if ((zx != ax && overlap(zx, bx, ax, bx)) || (zy != ay && overlap(zy, by, ay, by)) || overlap(zx, bx, zy, by) ||
        overlap(zx, bx, ay, by) || overlap(zy, by, ax, bx))
        return PSD_EINVAL;
    const size_t one = ((size_t)g.total * sizeof(cd) + 255) / 256 * 256;
    cd *b0 = static_cast<cd *>(ws), *b1 = reinterpret_cast<cd *>(static_cast<char *>(ws) + one);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (aff_adjoint(g, ay, ax, zx, b0, b1, s) != hipSuccess) return PSD_EDEVICE;
    if (aff_apply(g, zx, ay, zy, b0, b1, s) != hipSuccess) return PSD_EDEVICE;
    return PSD_OK;
}

}  // extern "C"
