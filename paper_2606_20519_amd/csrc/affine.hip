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
// nonzeros per row (s_alpha has 1, 2 or up to d entries).  Each direction is
// three memory-bound passes over the d^8 complex entries, each reading its
// input once into LDS: modes 2 and 3 of one D x D block of y together (with
// the svec unpack or pack), mode 1, and mode 0 (with the gather of the
// allowed coefficients to x by a closed-form rank, or the scatter from x).
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

// Nonzeros of the D rows of one local transform (dir 0: the forward rows
// gm_row, dir 1: the adjoint rows gm_col), tabulated in LDS by each
// workgroup.
struct AffTab {
    int j[64][8];
    cd c[64][8];
    int n[64];
};

__device__ __forceinline__ void aff_build_tab(AffTab &T, int d, int dir) {
    const int D = d * d;
    for (int r = threadIdx.x; r < D; r += blockDim.x) {
        int js[8];
        cd cs[8];
        const int c = dir ? gm_col(d, r, js, cs) : gm_row(d, r, js, cs);
        T.n[r] = c;
        for (int q = 0; q < c; ++q) {
            T.j[r][q] = js[q];
            T.c[r][q] = cs[q];
        }
    }
}

constexpr int AFF_T = 512;                 // threads per workgroup
constexpr int AFF_PER = 4096 / AFF_T;      // tile entries per thread (D^2 <= 4096, D x 64 <= 4096)

// Modes 2 and 3 of one slab T[p1, p2, :, :] (D^2 entries, contiguous in the
// tensor), which is the D x D block of y with rows a = (a1 d + a2) D + a_lo
// and columns b = (b1 d + b2) D + b_lo (p_m = a_m d + b_m; a_lo = a3 d + a4,
// b_lo = b3 d + b4).  dir 0: the block is read from the svec (upper rows,
// conjugated below the diagonal), transformed by the forward rows and
// written to the tensor.  dir 1: the tensor slab is transformed by the
// adjoint rows and its upper part written to the svec, y = base + result
// (base nullable); a block strictly below the diagonal is left to its
// mirror.  One workgroup per slab; the block stays in LDS (64 KiB at d = 8,
// two workgroups per CU), each mode's results staged in registers.
// Instance z of a batch (blockIdx.z) uses every pointer moved by z times its
// stride (elements); single calls pass zero strides.
// Per-instance strides of a batch (instance = grid z); an instance whose
// flag in `active` (nullable) is 0 is skipped.
struct AffStrides {
    int64_t y, t, base, yout;
    const int *active;
};

__global__ void __launch_bounds__(AFF_T) aff_slab_kernel(const double *__restrict__ ysv, const cd *__restrict__ tin,
                                                         cd *tout, const double *base, double *yout, int d, int dir,
                                                         AffStrides zs) {
    __shared__ cd S[4096];
    __shared__ AffTab tab;
    if (zs.active && !zs.active[blockIdx.z]) return;
    {
        const int64_t z = blockIdx.z;
        if (ysv) ysv += z * zs.y;
        if (tin) tin += z * zs.t;
        if (tout) tout += z * zs.t;
        if (base) base += z * zs.base;
        if (yout) yout += z * zs.yout;
    }
    const int D = d * d, n = D * D, DD = D * D;
    const int slab = blockIdx.x;
    const int p1 = slab / D, p2 = slab - p1 * D;
    const int a1 = p1 / d, b1 = p1 - a1 * d, a2 = p2 / d, b2 = p2 - a2 * d;
    const int A0 = (a1 * d + a2) * D, B0 = (b1 * d + b2) * D;
    const double rs2 = 0.70710678118654752440, rt2 = 1.41421356237309504880;
    aff_build_tab(tab, d, dir);
    const int tid = threadIdx.x;
    if (dir == 0) {
        for (int e = tid; e < DD; e += AFF_T) {
            // consecutive threads walk a stored svec row
            int al, bl;
            if (A0 > B0) { bl = e / D; al = e - bl * D; }
            else { al = e / D; bl = e - al * D; }
            const int a = A0 + al, b = B0 + bl;
            cd v;
            if (a == b) {
                v = cmk(ysv[svec_col_start(n, a)], 0.0);
            } else if (a < b) {
                const int64_t o = svec_off(n, b, a);
                v = cmk(ysv[o] * rs2, ysv[o + 1] * rs2);
            } else {
                const int64_t o = svec_off(n, a, b);
                v = cmk(ysv[o] * rs2, -ysv[o + 1] * rs2);
            }
            const int a3 = al / d, a4 = al - a3 * d, b3 = bl / d, b4 = bl - b3 * d;
            S[(a3 * d + b3) * D + (a4 * d + b4)] = v;
        }
    } else {
        for (int e = tid; e < DD; e += AFF_T) S[e] = tin[(int64_t)slab * DD + e];
    }
    __syncthreads();
    cd acc[AFF_PER];
#pragma unroll
    for (int k = 0; k < AFF_PER; ++k) {  // mode 3
        const int e = tid + k * AFF_T;
        acc[k] = cmk(0.0, 0.0);
        if (e < DD) {
            const int r = e / D, o = e - r * D;
            for (int q = 0; q < tab.n[o]; ++q) acc[k] = cfma(tab.c[o][q], S[r * D + tab.j[o][q]], acc[k]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < AFF_PER; ++k)
        if (tid + k * AFF_T < DD) S[tid + k * AFF_T] = acc[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < AFF_PER; ++k) {  // mode 2
        const int e = tid + k * AFF_T;
        acc[k] = cmk(0.0, 0.0);
        if (e < DD) {
            const int o = e / D, c = e - o * D;
            for (int q = 0; q < tab.n[o]; ++q) acc[k] = cfma(tab.c[o][q], S[tab.j[o][q] * D + c], acc[k]);
            if (dir == 0) tout[(int64_t)slab * DD + e] = acc[k];
        }
    }
    if (dir == 0 || A0 > B0) return;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < AFF_PER; ++k)
        if (tid + k * AFF_T < DD) S[tid + k * AFF_T] = acc[k];
    __syncthreads();
    for (int e = tid; e < DD; e += AFF_T) {
        const int al = e / D, bl = e - al * D;
        const int a = A0 + al, b = B0 + bl;
        if (a > b) continue;
        const int a3 = al / d, a4 = al - a3 * d, b3 = bl / d, b4 = bl - b3 * d;
        const cd v = S[(a3 * d + b3) * D + (a4 * d + b4)];
        if (a == b) {
            const int64_t o = svec_col_start(n, a);
            yout[o] = (base ? base[o] : 0.0) + v.x;
        } else {
            const int64_t o = svec_off(n, b, a);
            yout[o] = (base ? base[o] : 0.0) + rt2 * v.x;
            yout[o + 1] = (base ? base[o + 1] : 0.0) + rt2 * v.y;
        }
    }
}

// Mode m in {0, 1} of the tensor viewed as [H][D][R] (R = D^(3-m)): one
// workgroup per (h, 64 consecutive r), the D x 64 tile read once into LDS.
// Mode 0, dir 0 also gathers the allowed coefficients to x:
// x = -Re c (A^T y), or (a_x + Re c)/2 with a_x given; mode 0, dir 1 reads
// its input from x (coefficient -1 at the allowed indices, 0 elsewhere)
// instead of a tensor.
// Strides as for aff_slab_kernel: t for the tensors, x for x_in / a_x / x_out.
struct AffOuterStrides {
    int64_t t, x;
    const int *active;
};

__global__ void __launch_bounds__(AFF_T) aff_outer_kernel(const cd *__restrict__ tin, cd *tout,
                                                          const double *__restrict__ xin, const double *ax,
                                                          double *xout, int d, int m, int dir, AffOuterStrides zs) {
    __shared__ cd tile[64][64];
    __shared__ AffTab tab;
    if (zs.active && !zs.active[blockIdx.z]) return;
    {
        const int64_t z = blockIdx.z;
        if (tin) tin += z * zs.t;
        if (tout) tout += z * zs.t;
        if (xin) xin += z * zs.x;
        if (ax) ax += z * zs.x;
        if (xout) xout += z * zs.x;
    }
    const int D = d * d, DD = D * D;
    const int R = m == 0 ? DD * D : DD;
    const int ntr = (R + 63) / 64;
    const int h = blockIdx.x / ntr, r0 = (blockIdx.x - h * ntr) * 64;
    aff_build_tab(tab, d, dir);
    const int tid = threadIdx.x;
    for (int e = tid; e < D * 64; e += AFF_T) {
        const int j = e >> 6, r = e & 63;
        if (r0 + r >= R) continue;
        const unsigned t = (unsigned)(h * D + j) * (unsigned)R + (unsigned)(r0 + r);
        cd v;
        if (m == 0 && dir == 1) {
            const int64_t rk = mu_rank(D, (int)(t / DD), (int)(t % DD));
            v = rk < 0 ? cmk(0.0, 0.0) : cmk(-xin[rk], 0.0);
        } else {
            v = tin[t];
        }
        tile[j][r] = v;
    }
    __syncthreads();
    for (int e = tid; e < D * 64; e += AFF_T) {
        const int o = e >> 6, r = e & 63;
        if (r0 + r >= R) continue;
        cd acc = cmk(0.0, 0.0);
        for (int q = 0; q < tab.n[o]; ++q) acc = cfma(tab.c[o][q], tile[tab.j[o][q]][r], acc);
        const unsigned t = (unsigned)(h * D + o) * (unsigned)R + (unsigned)(r0 + r);
        if (m == 0 && dir == 0) {
            const int64_t rk = mu_rank(D, (int)(t / DD), (int)(t % DD));
            if (rk >= 0) xout[rk] = ax ? 0.5 * (ax[rk] + acc.x) : -acc.x;
        } else {
            tout[t] = acc;
        }
    }
}

int aff_outer_grid(const AffGeo &g, int m) {
    const int R = m == 0 ? g.D * g.D * g.D : g.D * g.D;
    return (m == 0 ? 1 : g.D) * ((R + 63) / 64);
}

// x = A^T y, or z_x = (a_x - A^T y)/2 when ax is given: modes 3 and 2 with
// the svec unpack, mode 1, mode 0 with the gather.  nb instances (grid z):
// y, a_x and x move by ys and xs elements per instance, the two tensors b0,
// b1 by ts elements.
hipError_t aff_adjoint(const AffGeo &g, const double *y, const double *ax, double *x, cd *b0, cd *b1, hipStream_t st,
                       int nb = 1, int64_t ys = 0, int64_t xs = 0, int64_t ts = 0, const int *act = nullptr) {
    hipLaunchKernelGGL(aff_slab_kernel, dim3(g.D * g.D, 1, nb), dim3(AFF_T), 0, st, y, (const cd *)nullptr, b0,
                       (const double *)nullptr, (double *)nullptr, g.d, 0, AffStrides{ys, ts, 0, 0, act});
    hipLaunchKernelGGL(aff_outer_kernel, dim3(aff_outer_grid(g, 1), 1, nb), dim3(AFF_T), 0, st, b0, b1,
                       (const double *)nullptr, (const double *)nullptr, (double *)nullptr, g.d, 1, 0,
                       AffOuterStrides{ts, 0, act});
    hipLaunchKernelGGL(aff_outer_kernel, dim3(aff_outer_grid(g, 0), 1, nb), dim3(AFF_T), 0, st, b1, (cd *)nullptr,
                       (const double *)nullptr, ax, x, g.d, 0, 0, AffOuterStrides{ts, xs, act});
    return hipGetLastError();
}

// y = base + A x (base nullable): mode 0 with the scatter, mode 1, modes 2
// and 3 with the svec pack; batched as aff_adjoint.
hipError_t aff_apply(const AffGeo &g, const double *x, const double *base, double *y, cd *b0, cd *b1, hipStream_t st,
                     int nb = 1, int64_t xs = 0, int64_t ys = 0, int64_t ts = 0, const int *act = nullptr) {
    hipLaunchKernelGGL(aff_outer_kernel, dim3(aff_outer_grid(g, 0), 1, nb), dim3(AFF_T), 0, st, (const cd *)nullptr,
                       b0, x, (const double *)nullptr, (double *)nullptr, g.d, 0, 1, AffOuterStrides{ts, xs, act});
    hipLaunchKernelGGL(aff_outer_kernel, dim3(aff_outer_grid(g, 1), 1, nb), dim3(AFF_T), 0, st, b0, b1,
                       (const double *)nullptr, (const double *)nullptr, (double *)nullptr, g.d, 1, 1,
                       AffOuterStrides{ts, 0, act});
    hipLaunchKernelGGL(aff_slab_kernel, dim3(g.D * g.D, 1, nb), dim3(AFF_T), 0, st, (const double *)nullptr, b1,
                       (cd *)nullptr, base, y, g.d, 1, AffStrides{0, ts, ys, ys, act});
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

// Batched forms for the SCS solver (one launch per pass for nb instances):
// instance z reads and writes its vectors ys / xs elements after instance
// 0's, and uses the two tensors of its workspace, wss bytes after instance
// 0's workspace (psd_affine_workspace_size bytes each).
hipError_t affine_step_batched(int d, const double *ax, const double *ay, double *zx, double *zy, int64_t xs,
                               int64_t ys, void *ws, int64_t wss, int nb, const int *active, hipStream_t st) {
    const AffGeo g = aff_geo(d);
    const size_t one = ((size_t)g.total * sizeof(cd) + 255) / 256 * 256;
    if (wss % (int64_t)sizeof(cd)) return hipErrorInvalidValue;
    cd *b0 = static_cast<cd *>(ws), *b1 = reinterpret_cast<cd *>(static_cast<char *>(ws) + one);
    const int64_t ts = wss / (int64_t)sizeof(cd);
    hipError_t e = aff_adjoint(g, ay, ax, zx, b0, b1, st, nb, ys, xs, ts, active);
    if (e != hipSuccess) return e;
    return aff_apply(g, zx, ay, zy, b0, b1, st, nb, xs, ys, ts, active);
}

hipError_t constraint_apply_batched(int d, const double *x, double *y, int64_t xs, int64_t ys, void *ws, int64_t wss,
                                    int nb, const int *active, hipStream_t st) {
    const AffGeo g = aff_geo(d);
    const size_t one = ((size_t)g.total * sizeof(cd) + 255) / 256 * 256;
    if (wss % (int64_t)sizeof(cd)) return hipErrorInvalidValue;
    cd *b0 = static_cast<cd *>(ws), *b1 = reinterpret_cast<cd *>(static_cast<char *>(ws) + one);
    return aff_apply(g, x, nullptr, y, b0, b1, st, nb, xs, ys, wss / (int64_t)sizeof(cd), active);
}

hipError_t constraint_adjoint_batched(int d, const double *y, double *x, int64_t ys, int64_t xs, void *ws,
                                      int64_t wss, int nb, const int *active, hipStream_t st) {
    const AffGeo g = aff_geo(d);
    const size_t one = ((size_t)g.total * sizeof(cd) + 255) / 256 * 256;
    if (wss % (int64_t)sizeof(cd)) return hipErrorInvalidValue;
    cd *b0 = static_cast<cd *>(ws), *b1 = reinterpret_cast<cd *>(static_cast<char *>(ws) + one);
    return aff_adjoint(g, y, nullptr, x, b0, b1, st, nb, ys, xs, wss / (int64_t)sizeof(cd), active);
}

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
