// Large-block FP64 path, stages after the tridiagonal eigensolver:
//  * select: count the eigenvalues > 0 (lambda ascending) and pick the side
//    with fewer columns, k = min(k+, k-);
//  * back-transform: V = Q Z for those k columns, four panels' reflectors
//    at a time (last group first): Z <- Z - V_g (T_g (V_g^H Z)), with V_g^H Z
//    as a split-K MFMA GEMM, the T_g product applied block by block from the
//    panels' factors and V_g^H V_g (T_g itself is never formed), and the
//    update as an MFMA GEMM (Z is read twice and written once per four
//    panels);
//  * reconstruction: Pi = V+ diag(lambda+) V+^H   (k+ <= k-), or
//    Pi = X - V- diag(lambda-) V-^H (otherwise), one MFMA GEMM over the
//    lower tiles whose epilogue writes the svec directly (App. D.2: zero the
//    negative eigenvalues of the eigendecomposition);
//  * the Daleckii-Krein derivative V (Gamma o (V^H G V)) V^H as four MFMA
//    GEMMs, Gamma applied in the epilogue of the second.
#include <algorithm>

#include "common.h"
#include "large.h"

namespace psd {

namespace {

constexpr int NB = LG_NB;
constexpr int BG = 4;           // panels per back-transform group
constexpr int GW = BG * NB;     // columns of a group's block reflector
static_assert(GW == 128, "bt_tw_kernel puts two columns of GW rows on 256 threads");
// Split-K chunk of V_b^H Z in the back-transform: 64 rows, more for large n
// so that the partial sums stay at most 16 (the GEMM has only NB rows, so
// the K split is where its parallelism comes from).
inline int kchunk_for(int n) { return std::max(64, (n + 16 * 64 - 1) / (16 * 64) * 64); }

inline size_t aup(size_t v) { return (v + 255) / 256 * 256; }

__global__ void init_status_kernel(int *ksel, int64_t zs) {
    ksel = member_ptr(ksel, zs, blockIdx.z);
    if (threadIdx.x < 4) ksel[threadIdx.x] = 0;
}

// k, sign, selected eigenvalues and the selected columns of Z (as complex).
__global__ void __launch_bounds__(256) select_kernel(const double *__restrict__ lam, const double *__restrict__ Z,
                                                     int n, int all_columns, double2 *Zc, int64_t lda,
                                                     double *lamsel, int *ksel, double *sgn,
                                                     psd_dev_info *info, int64_t zs, const int *infoidx) {
    {
        const int mb = blockIdx.z;
        lam = member_ptr(lam, zs, mb);
        Z = member_ptr(Z, zs, mb);
        Zc = member_ptr(Zc, zs, mb);
        lamsel = member_ptr(lamsel, zs, mb);
        ksel = member_ptr(ksel, zs, mb);
        sgn = member_ptr(sgn, zs, mb);
        if (info) info += infoidx ? infoidx[mb] : mb;
    }
    // first index with lambda > 0
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (lam[mid] > 0.0) hi = mid; else lo = mid + 1;
    }
    const int npos = n - lo, nneg = lo;
    int k, start;
    double s;
    if (all_columns) { k = n; start = 0; s = 1.0; }
    else if (npos <= nneg) { k = npos; start = n - npos; s = 1.0; }
    else { k = nneg; start = 0; s = -1.0; }
    const int c = blockIdx.y;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (c == 0 && r == 0) {
        ksel[0] = k;
        ksel[1] = npos;
        *sgn = s;
        if (info) {
            info->status = ksel[2];
            info->n_pos = npos;
            info->n_neg = nneg;
            info->iters = 0;
            info->fallback = 0;
            info->reserved = 0;
            info->est_rel_err = 0.0;
            info->scale = 0.0;
        }
    }
    if (c >= k || r >= n) return;
    Zc[r + (int64_t)c * lda] = cmk(Z[r + (int64_t)(start + c) * n], 0.0);
    if (r == 0) {
        const double l = lam[start + c];
        lamsel[c] = all_columns ? fmax(l, 0.0) : l;
    }
}

// Block reflector of a group of up to BG consecutive panels (reflector
// columns p0 .. p0 + G - 1): H_{b0} ... H_{b0+g-1} = I - V T V^H, where the
// two-block identity (I - V1 T1 V1^H)(I - V2 T2 V2^H)
//   = I - [V1 V2] [[T1, -T1 S12 T2], [0, T2]] [V1 V2]^H,   S = V^H V,
// extends to g blocks with T upper triangular.  T is never formed: Y = T W
// follows from the bottom block up, Y_j = T_j (W_j - sum_{l > j} S_jl Y_l).

// S = sum of the split-K partials of V^H V (entries above the diagonal
// blocks are the ones read).
__global__ void __launch_bounds__(256) s_reduce_kernel(const double2 *__restrict__ spart, int nz, int64_t szstride,
                                                       double2 *S, int64_t zs) {
    spart = member_ptr(spart, zs, blockIdx.z);
    S = member_ptr(S, zs, blockIdx.z);
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= GW * GW) return;
    double2 pz[16];  // nz <= 16: every partial in flight at once
#pragma unroll
    for (int z = 0; z < 16; ++z) pz[z] = z < nz ? spart[z * szstride + idx] : cmk(0.0, 0.0);
    double2 acc = cmk(0.0, 0.0);
#pragma unroll
    for (int z = 0; z < 16; ++z) acc = cadd(acc, pz[z]);
    for (int z = 16; z < nz; ++z) acc = cadd(acc, spart[z * szstride + idx]);
    S[idx] = acc;
}

// W2 = T W, W = sum_z partial_z (G rows, ld GW), for columns c < k: two
// columns per workgroup, the rows on the threads; T from the panels'
// factors Tp (NB x NB each) and S as above.
__global__ void __launch_bounds__(256) bt_tw_kernel(const double2 *__restrict__ wpart, int nz, int64_t zstride,
                                                    const double2 *__restrict__ Tp, const double2 *__restrict__ S,
                                                    int G, const int *ksel, double2 *W2, int64_t zs) {
    {
        const int mb = blockIdx.z;
        wpart = member_ptr(wpart, zs, mb);
        Tp = member_ptr(Tp, zs, mb);
        S = member_ptr(S, zs, mb);
        ksel = member_ptr(ksel, zs, mb);
        W2 = member_ptr(W2, zs, mb);
    }
    __shared__ double2 Wl[GW][3];  // W, then the block's right-hand side
    __shared__ double2 Yl[GW][3];  // Y
    const int t = threadIdx.x, i = t % GW, cl = t / GW;
    const int c = blockIdx.x * 2 + cl;
    const int k = ksel[0];
    const bool live = c < k && i < G;
    double2 acc = cmk(0.0, 0.0);
    if (live) {
        double2 pz[16];
#pragma unroll
        for (int z = 0; z < 16; ++z) pz[z] = z < nz ? wpart[z * zstride + i + (int64_t)c * GW] : cmk(0.0, 0.0);
#pragma unroll
        for (int z = 0; z < 16; ++z) acc = cadd(acc, pz[z]);
        for (int z = 16; z < nz; ++z) acc = cadd(acc, wpart[z * zstride + i + (int64_t)c * GW]);
    }
    Wl[i][cl] = acc;
    Yl[i][cl] = cmk(0.0, 0.0);
    __syncthreads();
    const int g = (G + NB - 1) / NB, bj = i / NB, r = i % NB;
    for (int j = g - 1; j >= 0; --j) {
        const int kbj = min(NB, G - j * NB);
        // right-hand side W_j - sum_{l > j} S_jl Y_l
        if (bj == j && live) {
            double2 rhs = Wl[i][cl];
#pragma unroll 8
            for (int m = (j + 1) * NB; m < G; ++m) rhs = csub(rhs, cmul(S[i + (int64_t)m * GW], Yl[m][cl]));
            Wl[i][cl] = rhs;
        }
        __syncthreads();
        // Y_j = T_j (right-hand side), T_j upper triangular
        if (bj == j && live) {
            const double2 *Tj = Tp + (int64_t)j * NB * NB;
            double2 y = cmk(0.0, 0.0);
#pragma unroll 8
            for (int m = r; m < kbj; ++m) y = cfma(Tj[r + (int64_t)m * NB], Wl[j * NB + m][cl], y);
            Yl[i][cl] = y;
        }
        __syncthreads();
    }
    if (live) W2[i + (int64_t)c * GW] = Yl[i][cl];
}

__global__ void __launch_bounds__(256) save_kernel(const double *__restrict__ lam, const double2 *__restrict__ Zc,
                                                   int64_t lda, int n, double *saved) {
    const int c = blockIdx.y;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    if (c == 0) saved[r] = lam[r];
    double2 *V = reinterpret_cast<double2 *>(saved + n);
    V[r + (int64_t)c * n] = Zc[r + (int64_t)c * lda];
}

// Full Hermitian matrix from an svec (for the derivative's cotangent).
__global__ void __launch_bounds__(256) unpack_full_kernel(const double *__restrict__ x, double2 *G, int64_t ld,
                                                          int n) {
    const int j = blockIdx.y;
    const int i = j + blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double rs2 = 0.70710678118654752440;
    if (i == j) {
        G[i + (int64_t)j * ld] = cmk(x[svec_col_start(n, j)], 0.0);
    } else {
        const int64_t o = svec_off(n, i, j);
        const double2 v = cmk(x[o] * rs2, x[o + 1] * rs2);
        G[i + (int64_t)j * ld] = v;
        G[j + (int64_t)i * ld] = cconj(v);
    }
}

// saved record -> eigenvalues and V (ld n) views are used directly; this
// copies V into the workspace layout when the caller passed `saved`.
__global__ void __launch_bounds__(256) load_saved_kernel(const double *__restrict__ saved, int n, double *lam,
                                                         double2 *Zc, int64_t lda) {
    const int c = blockIdx.y;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    if (c == 0) lam[r] = saved[r];
    const double2 *V = reinterpret_cast<const double2 *>(saved + n);
    Zc[r + (int64_t)c * lda] = V[r + (int64_t)c * n];
}

}  // namespace

size_t large_layout(int n, int flags, void *base, LargeWs *w) {
    size_t off = 0;
    char *b = static_cast<char *>(base);
    auto take = [&](size_t bytes) -> void * {
        void *p = b ? b + off : nullptr;
        off += aup(bytes);
        return p;
    };
    LargeWs L{};
    L.n = n;
    L.lda = (n + 63) / 64 * 64;
    L.mb = (n + LG_TILE - 1) / LG_TILE;
    L.npanel = (n - 1 + NB - 1) / NB;
    const bool full = (flags & 1) != 0;
    L.kmax = full ? n : n / 2 + 1;
    L.kchunk = kchunk_for(n);
    L.nchunk = (n + L.kchunk - 1) / L.kchunk;
    const size_t cdsz = sizeof(double2), dsz = sizeof(double);
    L.M = (double2 *)take(cdsz * L.lda * n);
    L.W = (double2 *)take(cdsz * L.lda * NB);
    L.vbuf = (double2 *)take(cdsz * L.lda);
    L.tau = (double2 *)take(cdsz * n);
    L.d = (double *)take(dsz * n);
    L.e = (double *)take(dsz * n);
    L.P = (double2 *)take(cdsz * (size_t)L.mb * L.mb * LG_TILE);
    L.tdot = (double *)take(dsz * (size_t)L.mb * (L.mb + 1) / 2);
    L.pq = (double2 *)take(cdsz * (size_t)L.mb * 2 * NB);
    L.npart = (double *)take(dsz * (size_t)L.mb);
    L.T = (double2 *)take(cdsz * (size_t)L.npanel * NB * NB);
    L.Q0 = (double *)take(dsz * (size_t)n * n);
    L.Q1 = (double *)take(dsz * (size_t)n * n);
    L.D0 = (double *)take(dsz * n);
    L.D1 = (double *)take(dsz * n);
    L.U = (double *)take(dsz * (size_t)n * n);
    L.dcd = (double *)take(dsz * (size_t)16 * n);
    L.dci = (int *)take(sizeof(int) * (size_t)8 * n);
    L.dcs = (int *)take(sizeof(int) * (size_t)4 * n);
    L.gdesc = (GemmDesc *)take(sizeof(GemmDesc) * (size_t)(n + 2));
    L.Zc = (double2 *)take(cdsz * L.lda * L.kmax);
    L.lamsel = (double *)take(dsz * L.kmax);
    L.wpart = (double *)take(cdsz * (size_t)L.nchunk * GW * L.kmax);
    L.W2 = (double2 *)take(cdsz * (size_t)GW * L.kmax);
    L.Sg = (double2 *)take(cdsz * (size_t)GW * GW);
    L.spart = (double2 *)take(cdsz * (size_t)L.nchunk * GW * GW);
    L.ksel = (int *)take(sizeof(int) * 4);
    L.sgn = (double *)take(dsz);
    L.B1 = full ? (double2 *)take(cdsz * (size_t)n * n) : nullptr;
    L.lam = L.D0;
    L.Zfinal = L.Q0;
    L.nmem = 1;
    L.zs = 0;
    L.ioff = nullptr;
    L.infoidx = nullptr;
    if (w) *w = L;
    return off;
}

hipError_t large_init(const LargeWs &w, hipStream_t st) {
    hipLaunchKernelGGL(init_status_kernel, dim3(1, 1, w.nmem), dim3(64), 0, st, w.ksel, w.zs);
    return hipGetLastError();
}

hipError_t large_select(const LargeWs &w, psd_dev_info *info, hipStream_t st, bool all_columns) {
    const int kcols = all_columns ? w.n : w.n / 2 + 1;
    dim3 grid((w.n + 255) / 256, std::min(kcols, w.kmax), w.nmem);
    hipLaunchKernelGGL(select_kernel, grid, dim3(256), 0, st, w.lam, w.Zfinal, w.n, all_columns ? 1 : 0, w.Zc,
                       w.lda, w.lamsel, w.ksel, w.sgn, info, w.zs, w.infoidx);
    return hipGetLastError();
}

hipError_t large_backtransform(const LargeWs &w, int ncols_max, hipStream_t st) {
    const int n = w.n;
    const int64_t zstride = (int64_t)GW * w.kmax, szstride = (int64_t)GW * GW;
    const int ngroup = (w.npanel + BG - 1) / BG;
    for (int gi = ngroup - 1; gi >= 0; --gi) {
        const int b0 = gi * BG, b1 = std::min(w.npanel, b0 + BG), g = b1 - b0;
        const int p0 = b0 * NB;
        const int G = std::min(n - 1, b1 * NB) - p0;  // reflector columns of the group
        const int mr = n - 1 - p0;
        const double2 *Vg = w.M + (p0 + 1) + (int64_t)p0 * w.lda;
        hipError_t e;
        // S = V^H V (its blocks above the diagonal couple the panels)
        if (g > 1) {
            GemmDesc sg{};
            sg.M = sg.N = G; sg.K = mr;
            sg.A = GemmOperand{Vg, Vg, w.lda, w.lda, mr, OP_C, nullptr};
            sg.B = GemmOperand{Vg, Vg, w.lda, w.lda, mr, OP_N, nullptr};
            sg.C = w.spart; sg.ldc = GW; sg.alpha = 1.0; sg.beta = 0.0;
            sg.kchunk = w.kchunk; sg.c_zstride = szstride;
            sg.nmem = w.nmem; sg.zs = w.zs;
            if ((e = gemm_launch(sg, true, EPI_STORE, st)) != hipSuccess) return e;
            hipLaunchKernelGGL(s_reduce_kernel, dim3(GW * GW / 256, 1, w.nmem), dim3(256), 0, st,
                               reinterpret_cast<const double2 *>(w.spart), gemm_kslices(sg), szstride, w.Sg, w.zs);
        }
        // partials of V^H Z over row chunks
        GemmDesc gm{};
        gm.M = G; gm.N = ncols_max; gm.K = mr;
        gm.A = GemmOperand{Vg, Vg, w.lda, w.lda, mr, OP_C, nullptr};
        gm.B = GemmOperand{w.Zc + (p0 + 1), w.Zc + (p0 + 1), w.lda, w.lda, mr, OP_N, nullptr};
        gm.C = w.wpart; gm.ldc = GW; gm.alpha = 1.0; gm.beta = 0.0;
        gm.dN = w.ksel;
        gm.kchunk = w.kchunk; gm.c_zstride = zstride;
        gm.nmem = w.nmem; gm.zs = w.zs;
        if ((e = gemm_launch(gm, true, EPI_STORE, st)) != hipSuccess) return e;
        const int nz = gemm_kslices(gm);
        hipLaunchKernelGGL(bt_tw_kernel, dim3((ncols_max + 1) / 2, 1, w.nmem), dim3(256), 0, st,
                           reinterpret_cast<const double2 *>(w.wpart), nz, zstride, w.T + (int64_t)b0 * NB * NB, w.Sg,
                           G, w.ksel, w.W2, w.zs);
        // Z[p0+1:, :] -= V W2
        GemmDesc u{};
        u.M = mr; u.N = ncols_max; u.K = G;
        u.A = GemmOperand{Vg, Vg, w.lda, w.lda, G, OP_N, nullptr};
        u.B = GemmOperand{w.W2, w.W2, GW, GW, G, OP_N, nullptr};
        u.C = w.Zc + (p0 + 1); u.ldc = w.lda; u.alpha = -1.0; u.beta = 1.0;
        u.dN = w.ksel;
        u.nmem = w.nmem; u.zs = w.zs;
        if ((e = gemm_launch(u, true, EPI_STORE, st)) != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t large_reconstruct(const LargeWs &w, const double *x, double *y, int kmax, hipStream_t st) {
    GemmDesc g{};
    g.M = g.N = w.n;
    g.K = kmax;
    g.lower_only = 1;
    g.A = GemmOperand{w.Zc, w.Zc, w.lda, w.lda, kmax, OP_N, w.lamsel};
    g.B = GemmOperand{w.Zc, w.Zc, w.lda, w.lda, kmax, OP_C, nullptr};
    g.y = y; g.xbase = x; g.svec_n = w.n; g.sign = 1.0;
    g.dsign = w.sgn;
    g.dK = w.ksel;
    g.dstatus = w.ksel + 2;
    g.nmem = w.nmem; g.zs = w.zs; g.ioff = w.ioff;
    return gemm_launch(g, true, EPI_SVEC, st);
}

hipError_t large_save(const LargeWs &w, double *saved, hipStream_t st) {
    dim3 grid((w.n + 255) / 256, w.n);
    hipLaunchKernelGGL(save_kernel, grid, dim3(256), 0, st, w.lam, w.Zc, w.lda, w.n, saved);
    return hipGetLastError();
}

// gx = svec(V (Gamma o (V^H G V)) V^H), V = Zc (n x n, ld lda), lambda = w.lam.
hipError_t large_vjp_from_v(const LargeWs &w, const double *gy, double *gx, hipStream_t st) {
    const int n = w.n;
    double2 *G = w.M;   // cotangent (full Hermitian), later Gamma o (V^H G V)
    double2 *B1 = w.B1;
    dim3 grid((n + 255) / 256, n);
    hipLaunchKernelGGL(unpack_full_kernel, grid, dim3(256), 0, st, gy, G, w.lda, n);
    // B1 = G V   (ld n)
    GemmDesc a{};
    a.M = a.N = a.K = n;
    a.A = GemmOperand{G, G, w.lda, w.lda, n, OP_N, nullptr};
    a.B = GemmOperand{w.Zc, w.Zc, w.lda, w.lda, n, OP_N, nullptr};
    a.C = B1; a.ldc = n; a.alpha = 1.0; a.beta = 0.0;
    hipError_t e = gemm_launch(a, true, EPI_STORE, st);
    if (e != hipSuccess) return e;
    // G = Gamma o (V^H B1)   (reuse G's storage, ld lda)
    GemmDesc b{};
    b.M = b.N = b.K = n;
    b.A = GemmOperand{w.Zc, w.Zc, w.lda, w.lda, n, OP_C, nullptr};
    b.B = GemmOperand{B1, B1, n, n, n, OP_N, nullptr};
    b.C = G; b.ldc = w.lda; b.alpha = 1.0; b.beta = 0.0;
    b.lam = w.lam;
    e = gemm_launch(b, true, EPI_GAMMA, st);
    if (e != hipSuccess) return e;
    // B1 = G V^H
    GemmDesc c{};
    c.M = c.N = c.K = n;
    c.A = GemmOperand{G, G, w.lda, w.lda, n, OP_N, nullptr};
    c.B = GemmOperand{w.Zc, w.Zc, w.lda, w.lda, n, OP_C, nullptr};
    c.C = B1; c.ldc = n; c.alpha = 1.0; c.beta = 0.0;
    e = gemm_launch(c, true, EPI_STORE, st);
    if (e != hipSuccess) return e;
    // gx = svec(V B1), lower tiles
    GemmDesc d{};
    d.M = d.N = d.K = n;
    d.lower_only = 1;
    d.A = GemmOperand{w.Zc, w.Zc, w.lda, w.lda, n, OP_N, nullptr};
    d.B = GemmOperand{B1, B1, n, n, n, OP_N, nullptr};
    d.y = gx; d.xbase = nullptr; d.svec_n = n; d.sign = 1.0;
    d.dstatus = w.ksel + 2;
    return gemm_launch(d, true, EPI_SVEC, st);
}

hipError_t large_load_saved(const LargeWs &w, const double *saved, hipStream_t st) {
    dim3 grid((w.n + 255) / 256, w.n);
    hipLaunchKernelGGL(load_saved_kernel, grid, dim3(256), 0, st, saved, w.n, w.D0, w.Zc, w.lda);
    return hipGetLastError();
}

}  // namespace psd
