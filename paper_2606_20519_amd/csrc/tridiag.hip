// Blocked Householder reduction of a Hermitian matrix (order n > 64) to real
// symmetric tridiagonal form, M = Q T Q^H, Q = H_0 H_1 ... H_{n-2},
// H_j = I - tau_j v_j v_j^H (v_j(j+1) = 1, zero above), on the lower triangle
// of M stored column-major in HBM.
//
// Columns are processed in panels of NB.  Inside a panel the trailing matrix
// is not touched; column j sees the panel's earlier reflectors through
//   A_cur = A - V W^H - W V^H                     (V, W: panel columns so far)
// and the new w_j follows from one Hermitian matrix-vector product with the
// stored (not yet updated) trailing matrix:
//   y = A v,  p = V^H v,  q = W^H v,  u = y - V q - W p,
//   w = tau u - 1/2 |tau|^2 (v^H A v - 2 Re q^H p) v.
// After the panel, the trailing matrix gets the rank-2NB update
// A -= V W^H + W V^H as one FP64 MFMA GEMM (lower tiles only).
//
// Per column two launches: the tiled HEMV over the lower triangle (one
// workgroup per 64x64 tile; each first rebuilds the column's reflector from
// the sigma partials, identically), and the w/next-column step (one workgroup
// per 64 rows), which also extends the block-reflector factor T and leaves
// the next column's sigma partials.  Partial sums go to fixed slots, no
// atomics: the result is deterministic.  Only the lower triangle (row >=
// column) of M is ever read.
#include "common.h"
#include "large.h"
#include "timing.h"

namespace psd {

namespace {

constexpr int TT = LG_TILE;
constexpr int NB = LG_NB;

// svec -> lower triangle of M (M = conj X, see common.h); flags non-finite.
__global__ void __launch_bounds__(256) unpack_kernel(const double *__restrict__ x, double2 *M, int64_t lda, int n,
                                                     int *status) {
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
    }
    if (!(isfinite(v.x) && isfinite(v.y))) status[2] = ST_ENONFINITE;
    M[i + j * lda] = v;
}

// Reflector of column j from alpha = M(j+1, j) and sigma = sum_{r > j+1}
// |M(r, j)|^2: H = I - tau v v^H with H^H [alpha; x] = [beta; 0], beta real,
// v = [1; x / (alpha - beta)].  Every caller gets bitwise the same values.
struct Refl {
    double2 tau, scale;
    double beta;
};
__device__ __forceinline__ Refl make_refl(double2 alpha, double sigma) {
    Refl h;
    if (sigma == 0.0 && alpha.y == 0.0) {
        h.tau = cmk(0.0, 0.0); h.beta = alpha.x; h.scale = cmk(0.0, 0.0);
    } else {
        h.beta = -copysign(sqrt(cabs2(alpha) + sigma), alpha.x);
        h.tau = cmk((h.beta - alpha.x) / h.beta, -alpha.y / h.beta);
        h.scale = cdiv(cmk(1.0, 0.0), cmk(alpha.x - h.beta, alpha.y));
    }
    return h;
}

// sigma partial of column j (first column of a panel): rows > j+1.
__global__ void __launch_bounds__(512) norm_kernel(const double2 *__restrict__ M, int64_t lda, int n, int j,
                                                   double *npart) {
    __shared__ double red[16];
    const double2 *col = M + (int64_t)j * lda;
    double part = 0.0;
    for (int r = j + 2 + threadIdx.x; r < n; r += blockDim.x) part += cabs2(col[r]);
    const double sum = block_sum(part, red);
    if (threadIdx.x == 0) npart[0] = sum;
}

// Last diagonal entry of T.
__global__ void final_kernel(const double2 *__restrict__ M, int64_t lda, int n, double *d) {
    if (threadIdx.x == 0) d[n - 1] = M[(n - 1) + (int64_t)(n - 1) * lda].x;
}

// Reflector of column j (recomputed identically by every workgroup from the
// sigma partials), then tile (I, J), J <= I, of the trailing matrix
// A = M[s:, s:] (s = j+1) times v:
//   direct part  A_IJ v_J      -> P[I][slot J]
//   adjoint part A_IJ^H v_I    -> P[J][slot I]     (I > J only)
//   tdot[tile]  = w * Re(v_I^H A_IJ v_J), w = 1 (diagonal) or 2
// Diagonal-tile workgroups write v for their rows into vbuf and produce
// p = V^H v and q = W^H v over their 64 rows for the c panel columns done.
__global__ void __launch_bounds__(256) hemv_kernel(const double2 *__restrict__ M, int64_t lda, int n, int j,
                                                   int mt, const double *__restrict__ npart, int nparts,
                                                   double2 *vbuf, const double2 *__restrict__ W, int p0, int c,
                                                   double2 *P, double *tdot, double2 *pq, double2 *taus,
                                                   double *d, double *e) {
    __shared__ double2 tile[TT * (TT + 1)];
    __shared__ double2 vI[TT], vJ[TT];
    __shared__ double2 rowp[4][TT], colp[4][TT];
    const int s = j + 1;
    const int b = blockIdx.x;
    int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= b) ++I;
    while (I * (I + 1) / 2 > b) --I;
    const int J = b - I * (I + 1) / 2;
    const int t = threadIdx.x, lane = t & 63, g = t >> 6;
    const int r0 = s + I * TT, c0 = s + J * TT;
    const double2 *colj = M + (int64_t)j * lda;
    // sigma: every wave reduces the same partials in the same lane order
    double sp = 0.0;
    for (int k = lane; k < nparts; k += 64) sp += npart[k];
    const double sigma = warp_sum(sp);
    const Refl h = make_refl(colj[s], sigma);
    {
        const bool rowok = r0 + lane < n;
#pragma unroll
        for (int cc = g; cc < TT; cc += 4) {
            const int col = c0 + cc;
            double2 v = cmk(0.0, 0.0);
            if (rowok && col < n && (I != J || lane >= cc)) v = M[(r0 + lane) + (int64_t)col * lda];
            tile[cc * (TT + 1) + lane] = v;
        }
        if (t < 2 * TT) {
            const int row = (t < TT ? r0 : c0) + lane;
            double2 v = cmk(0.0, 0.0);
            if (row == s) v = cmk(1.0, 0.0);
            else if (row < n) v = cmul(colj[row], h.scale);
            if (t < TT) vI[t] = v; else vJ[t - TT] = v;
        }
    }
    __syncthreads();
    if (b == 0 && t == 0) {
        d[j] = colj[j].x;
        e[j] = h.beta;
        taus[j] = h.tau;
    }
    // partial row sums (direct) and column sums (adjoint) over 16-wide strips
    {
        double2 racc = cmk(0.0, 0.0), cacc = cmk(0.0, 0.0);
        const int k0 = 16 * g;
        if (I == J) {
#pragma unroll 4
            for (int cc = k0; cc < k0 + 16; ++cc) {
                double2 a;
                if (cc < lane) a = tile[cc * (TT + 1) + lane];
                else if (cc == lane) a = cmk(tile[cc * (TT + 1) + lane].x, 0.0);
                else a = cconj(tile[lane * (TT + 1) + cc]);
                racc = cfma(a, vI[cc], racc);
            }
        } else {
#pragma unroll 4
            for (int cc = k0; cc < k0 + 16; ++cc) racc = cfma(tile[cc * (TT + 1) + lane], vJ[cc], racc);
#pragma unroll 4
            for (int rr = k0; rr < k0 + 16; ++rr) cacc = cfmac(tile[lane * (TT + 1) + rr], vI[rr], cacc);
        }
        rowp[g][lane] = racc;
        colp[g][lane] = cacc;
    }
    // diagonal tiles: p = V^H v, q = W^H v over these rows, 2c columns,
    // column cc on wave cc % 4 with the 64 rows on the lanes
    if (I == J && c > 0) {
        const bool ok = r0 + lane < n;
        const double2 vl = vI[lane];
        for (int q = g; q < 2 * c; q += 4) {
            const bool isv = q < c;
            const int cc = isv ? q : q - c;
            const double2 *col = isv ? (M + (int64_t)(p0 + cc) * lda) : (W + (int64_t)cc * lda);
            const double2 x = ok ? col[r0 + lane] : cmk(0.0, 0.0);
            const double2 pr = cmulc(x, vl);
            const double re = warp_sum(pr.x), im = warp_sum(pr.y);
            if (lane == 0) pq[((int64_t)I * 2 + (isv ? 0 : 1)) * NB + cc] = cmk(re, im);
        }
    }
    __syncthreads();
    if (t < TT) {
        const double2 y = cadd(cadd(rowp[0][t], rowp[1][t]), cadd(rowp[2][t], rowp[3][t]));
        P[((int64_t)I * mt + J) * TT + t] = y;
        if (I == J && r0 + t < n) vbuf[r0 + t] = vI[t];
        const double dv = warp_sum(cmulc(vI[t], y).x);
        if (t == 0) tdot[b] = (I == J) ? dv : 2.0 * dv;
    } else if (t < 2 * TT && I != J) {
        const int cc = t - TT;
        const double2 z = cadd(cadd(colp[0][cc], colp[1][cc]), cadd(colp[2][cc], colp[3][cc]));
        P[((int64_t)J * mt + I) * TT + cc] = z;
    }
}

// Rows of block I (64 rows from s): stores v into the reflector column j,
// w = tau u + a2 v into W[:, c] with u = y - V q - W p, and -- when column
// j+1 belongs to the same panel -- applies the panel update to column j+1 and
// writes its sigma partial (rows > j+2).  Workgroup 0 also appends column c
// of the block-reflector factor: T(c,c) = tau, T(0:c,c) = -tau T(0:c,0:c) p,
// since p = V^H v_c = G(0:c, c) for v_c vanishing above row j+1.
__global__ void __launch_bounds__(256) w_kernel(double2 *M, int64_t lda, int n, int j, int mt, int nt,
                                                const double2 *__restrict__ vbuf, double2 *W, int p0, int c,
                                                int next_in_panel, const double2 *__restrict__ P,
                                                const double *__restrict__ tdot, const double2 *__restrict__ pq,
                                                const double2 *__restrict__ taus, double2 *Tb, double *npart) {
    __shared__ double2 pS[NB], qS[NB], Ws[NB], Vs[NB];
    __shared__ double2 Tl[NB][NB + 1];
    __shared__ double red[8];
    __shared__ double2 ypart[4][TT], upart[4][TT], apart[4][TT];
    __shared__ double2 wsh;
    const int s = j + 1;
    const int I = blockIdx.x, t = threadIdx.x;
    const int r = t & 63, g = t >> 6;
    const int row = s + I * TT + r;
    const double2 tj = taus[j];
    // p = V^H v, q = W^H v: column q on wave q % 4, row blocks on the lanes
    for (int q = g; q < 2 * c; q += 4) {
        const bool isv = q < c;
        const int cc = isv ? q : q - c;
        double2 acc = cmk(0.0, 0.0);
        for (int bb = r; bb < mt; bb += 64) acc = cadd(acc, pq[((int64_t)bb * 2 + (isv ? 0 : 1)) * NB + cc]);
        const double re = warp_sum(acc.x), im = warp_sum(acc.y);
        if (r == 0) { if (isv) pS[cc] = cmk(re, im); else qS[cc] = cmk(re, im); }
    }
    if (next_in_panel && t >= 64 && t < 64 + c) {
        Ws[t - 64] = W[s + (int64_t)(t - 64) * lda];
        Vs[t - 64] = M[s + (int64_t)(p0 + t - 64) * lda];
    }
    if (I == 0)
        for (int idx = t; idx < c * c; idx += blockDim.x) Tl[idx % c][idx / c] = Tb[(idx % c) + (idx / c) * NB];
    double part = 0.0;
    for (int bb = t; bb < nt; bb += blockDim.x) part += tdot[bb];
    const double vAv = block_sum(part, red);  // barriers: pS/qS/Ws/Vs/Tl visible after it
    double qp = 0.0;
    for (int cc = 0; cc < c; ++cc) qp += cmulc(qS[cc], pS[cc]).x;
    const double a2 = -0.5 * cabs2(tj) * (vAv - 2.0 * qp);
    // block-reflector factor, column c
    if (I == 0 && t <= c) {
        double2 out;
        if (t == c) {
            out = tj;
        } else {
            double2 z = cmk(0.0, 0.0);
            for (int l = t; l < c; ++l) z = cfma(Tl[t][l], pS[l], z);
            out = cscale(cmul(tj, z), -1.0);
        }
        Tb[t + c * NB] = out;
    }
    // y, V q + W p and (for column j+1) the panel terms, split over 4 groups
    {
        double2 y = cmk(0.0, 0.0), u = cmk(0.0, 0.0), a = cmk(0.0, 0.0);
#pragma unroll 4
        for (int sl = g; sl < mt; sl += 4) y = cadd(y, P[((int64_t)I * mt + sl) * TT + r]);
        if (row < n) {
#pragma unroll 4
            for (int cc = g; cc < c; cc += 4) {
                const double2 vr = M[row + (int64_t)(p0 + cc) * lda];
                const double2 wr = W[row + (int64_t)cc * lda];
                u = cfma(vr, qS[cc], u);
                u = cfma(wr, pS[cc], u);
                if (next_in_panel) {
                    a = cfma(vr, cconj(Ws[cc]), a);
                    a = cfma(wr, cconj(Vs[cc]), a);
                }
            }
        }
        ypart[g][r] = y;
        upart[g][r] = u;
        apart[g][r] = a;
    }
    // w at row s, needed by every block for column j+1 (wave 0)
    if (next_in_panel && g == 0) {
        double2 ys = cmk(0.0, 0.0);
        for (int sl = r; sl < mt; sl += 64) ys = cadd(ys, P[(int64_t)sl * TT + 0]);
        ys = cmk(warp_sum(ys.x), warp_sum(ys.y));
        if (r == 0) {
            for (int cc = 0; cc < c; ++cc) {
                ys = csub(ys, cmul(Vs[cc], qS[cc]));
                ys = csub(ys, cmul(Ws[cc], pS[cc]));
            }
            wsh = cadd(cmul(tj, ys), cmk(a2, 0.0));  // v[s] = 1
        }
    }
    __syncthreads();
    double nrm = 0.0;
    if (t < TT && row < n) {
        const double2 y = cadd(cadd(ypart[0][r], ypart[1][r]), cadd(ypart[2][r], ypart[3][r]));
        const double2 vq = cadd(cadd(upart[0][r], upart[1][r]), cadd(upart[2][r], upart[3][r]));
        const double2 v = vbuf[row];
        M[row + (int64_t)j * lda] = v;
        const double2 w = cfma(cmk(a2, 0.0), v, cmul(tj, csub(y, vq)));
        W[row + (int64_t)c * lda] = w;
        if (next_in_panel) {
            // column j+1 of A_cur = A - V W^H - W V^H over panel columns 0..c
            const double2 pa = cadd(cadd(apart[0][r], apart[1][r]), cadd(apart[2][r], apart[3][r]));
            double2 a = csub(M[row + (int64_t)(j + 1) * lda], pa);
            a = csub(a, cmul(v, cconj(wsh)));
            a = csub(a, w);  // W(row,c) conj(V(s,c)), V(s,c) = 1
            M[row + (int64_t)(j + 1) * lda] = a;
            if (row > j + 2) nrm = cabs2(a);
        }
    }
    if (next_in_panel) {
        const double sum = block_sum(nrm, red);
        if (t == 0) npart[I] = sum;
    }
}

// Zero the upper triangle (incl. diagonal) of the reflector columns so that
// column j of M is exactly v_j (v_j(j+1) = 1 is already stored).
__global__ void __launch_bounds__(256) clean_kernel(double2 *M, int64_t lda, int n) {
    const int j = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i > j || j >= n) return;
    M[i + (int64_t)j * lda] = cmk(0.0, 0.0);
}

}  // namespace

hipError_t large_unpack(const LargeWs &w, const double *x, hipStream_t st) {
    dim3 grid((w.n + 255) / 256, w.n);
    hipLaunchKernelGGL(unpack_kernel, grid, dim3(256), 0, st, x, w.M, w.lda, w.n, w.ksel);
    return hipGetLastError();
}

hipError_t large_tridiag(const LargeWs &w, hipStream_t st) {
    const int n = w.n;
    for (int p0 = 0; p0 < n - 1; p0 += NB) {
        const int kb = min(NB, n - 1 - p0);
        double2 *Tb = w.T + (int64_t)(p0 / NB) * NB * NB;
        hipLaunchKernelGGL(norm_kernel, dim3(1), dim3(512), 0, st, w.M, w.lda, n, p0, w.npart);
        int nparts = 1;
        for (int c = 0; c < kb; ++c) {
            const int j = p0 + c, m = n - j - 1;
            const int mt = (m + TT - 1) / TT, nt = mt * (mt + 1) / 2;
            const int slot = timing_begin(KF_HEMV, st);
            hipLaunchKernelGGL(hemv_kernel, dim3(nt), dim3(256), 0, st, w.M, w.lda, n, j, mt, w.npart, nparts,
                               w.vbuf, w.W, p0, c, w.P, w.tdot, w.pq, w.tau, w.d, w.e);
            timing_end(slot, st, 8.0 * (double)m * (double)(m + 1));
            const int next_in_panel = (c + 1 < kb) ? 1 : 0;
            hipLaunchKernelGGL(w_kernel, dim3(mt), dim3(256), 0, st, w.M, w.lda, n, j, mt, nt, w.vbuf, w.W, p0,
                               c, next_in_panel, w.P, w.tdot, w.pq, w.tau, Tb, w.npart);
            nparts = mt;
        }
        const int t0 = p0 + kb;
        if (t0 < n) {
            GemmDesc g{};
            g.M = g.N = n - t0;
            g.K = 2 * kb;
            g.lower_only = 1;
            g.A = GemmOperand{w.M + t0 + (int64_t)p0 * w.lda, w.W + t0, w.lda, w.lda, kb, OP_N, nullptr};
            g.B = GemmOperand{w.W + t0, w.M + t0 + (int64_t)p0 * w.lda, w.lda, w.lda, kb, OP_C, nullptr};
            g.C = w.M + t0 + (int64_t)t0 * w.lda;
            g.ldc = w.lda;
            g.alpha = -1.0;
            g.beta = 1.0;
            hipError_t e = gemm_launch(g, true, EPI_STORE, st);
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL(final_kernel, dim3(1), dim3(64), 0, st, w.M, w.lda, n, w.d);
    return hipGetLastError();
}

hipError_t large_compute_T(const LargeWs &w, hipStream_t st) {
    dim3 grid((w.n + 255) / 256, w.n);
    hipLaunchKernelGGL(clean_kernel, grid, dim3(256), 0, st, w.M, w.lda, w.n);
    return hipGetLastError();
}

}  // namespace psd
