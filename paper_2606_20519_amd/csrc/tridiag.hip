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
// Per column three launches: reflector (1 workgroup), tiled HEMV over the
// lower triangle (one workgroup per 64x64 tile, partial sums per slot, no
// atomics: deterministic), and the w/next-column step (one workgroup per 64
// rows).  Only the lower triangle (row >= column) of M is ever read.
#include "common.h"
#include "large.h"

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

// Householder vector of column j: v = [1, x/(alpha - beta)], beta real.
__global__ void __launch_bounds__(512) refl_kernel(double2 *M, int64_t lda, int n, int j, double2 *vbuf,
                                                   double2 *tau, double *d, double *e) {
    __shared__ double red[16];
    const int t = threadIdx.x;
    if (j == n - 1) {
        if (t == 0) d[j] = M[j + j * lda].x;
        return;
    }
    const int s = j + 1;
    double2 *col = M + j * lda;
    double part = 0.0;
    for (int r = s + 1 + t; r < n; r += blockDim.x) part += cabs2(col[r]);
    const double sigma = block_sum(part, red);
    const double2 alpha = col[s];
    double2 tj, scale;
    double beta;
    if (sigma == 0.0 && alpha.y == 0.0) {
        tj = cmk(0.0, 0.0); beta = alpha.x; scale = cmk(0.0, 0.0);
    } else {
        beta = -copysign(sqrt(cabs2(alpha) + sigma), alpha.x);
        tj = cmk((beta - alpha.x) / beta, -alpha.y / beta);
        scale = cdiv(cmk(1.0, 0.0), cmk(alpha.x - beta, alpha.y));
    }
    for (int r = s + 1 + t; r < n; r += blockDim.x) {
        const double2 v = cmul(col[r], scale);
        col[r] = v;
        vbuf[r] = v;
    }
    if (t == 0) {
        col[s] = cmk(1.0, 0.0);
        vbuf[s] = cmk(1.0, 0.0);
        d[j] = col[j].x;
        e[j] = beta;
        tau[j] = tj;
    }
}

// Tile (I, J), J <= I, of the trailing matrix A = M[s:, s:] times v.
//   direct part  A_IJ v_J      -> P[I][slot J]
//   adjoint part A_IJ^H v_I    -> P[J][slot I]     (I > J only)
//   tdot[tile]  = w * Re(v_I^H A_IJ v_J), w = 1 (diagonal) or 2
// Diagonal-tile workgroups also produce p = V^H v and q = W^H v over their
// 64 rows for the c panel columns already done.
__global__ void __launch_bounds__(256) hemv_kernel(const double2 *__restrict__ M, int64_t lda, int n, int s,
                                                   int mt, const double2 *__restrict__ vbuf,
                                                   const double2 *__restrict__ W, int p0, int c, double2 *P,
                                                   double *tdot, double2 *pq) {
    __shared__ double2 tile[TT * (TT + 1)];
    __shared__ double2 vI[TT], vJ[TT];
    const int b = blockIdx.x;
    int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= b) ++I;
    while (I * (I + 1) / 2 > b) --I;
    const int J = b - I * (I + 1) / 2;
    const int t = threadIdx.x;
    const int r0 = s + I * TT, c0 = s + J * TT;
    {
        const int r = t & 63;
        const bool rowok = r0 + r < n;
        for (int cc = t >> 6; cc < TT; cc += 4) {
            const int col = c0 + cc;
            double2 v = cmk(0.0, 0.0);
            if (rowok && col < n && (I != J || r >= cc)) v = M[(r0 + r) + (int64_t)col * lda];
            tile[cc * (TT + 1) + r] = v;
        }
        if (t < TT) vI[t] = (r0 + t < n) ? vbuf[r0 + t] : cmk(0.0, 0.0);
        else if (t < 2 * TT) vJ[t - TT] = (c0 + t - TT < n) ? vbuf[c0 + t - TT] : cmk(0.0, 0.0);
    }
    __syncthreads();
    if (I == J) {
        if (t < TT) {
            // Hermitian tile from its lower triangle
            double2 acc = cmk(0.0, 0.0);
            for (int cc = 0; cc < TT; ++cc) {
                double2 a;
                if (cc < t) a = tile[cc * (TT + 1) + t];
                else if (cc == t) a = cmk(tile[cc * (TT + 1) + t].x, 0.0);
                else a = cconj(tile[t * (TT + 1) + cc]);
                acc = cfma(a, vI[cc], acc);
            }
            P[((int64_t)I * mt + I) * TT + t] = acc;
            const double dv = warp_sum(cmulc(vI[t], acc).x);
            if (t == 0) tdot[b] = dv;
        } else if (t >= 64 && t < 64 + 2 * c) {
            const int q = t - 64;
            const bool isv = q < c;
            const int cc = isv ? q : q - c;
            const double2 *col = isv ? (M + (int64_t)(p0 + cc) * lda) : (W + (int64_t)cc * lda);
            double2 acc = cmk(0.0, 0.0);
            for (int r = 0; r < TT && r0 + r < n; ++r) acc = cfmac(col[r0 + r], vI[r], acc);
            pq[((int64_t)I * 2 + (isv ? 0 : 1)) * NB + cc] = acc;
        }
    } else {
        if (t < TT) {
            double2 acc = cmk(0.0, 0.0);
            for (int cc = 0; cc < TT; ++cc) acc = cfma(tile[cc * (TT + 1) + t], vJ[cc], acc);
            P[((int64_t)I * mt + J) * TT + t] = acc;
            const double dv = warp_sum(cmulc(vI[t], acc).x);
            if (t == 0) tdot[b] = 2.0 * dv;
        } else if (t < 2 * TT) {
            const int cc = t - TT;
            double2 acc = cmk(0.0, 0.0);
            for (int r = 0; r < TT; ++r) acc = cfmac(tile[cc * (TT + 1) + r], vI[r], acc);
            P[((int64_t)J * mt + I) * TT + cc] = acc;
        }
    }
}

// w for rows of block I, stored in W[:, c]; if the next column is in the same
// panel, also applies the panel update to column j+1 (rows of block I).
__global__ void __launch_bounds__(256) w_kernel(double2 *M, int64_t lda, int n, int j, int s, int mt, int nt,
                                                const double2 *__restrict__ vbuf, double2 *W, int p0, int c,
                                                int next_in_panel, const double2 *__restrict__ P,
                                                const double *__restrict__ tdot, const double2 *__restrict__ pq,
                                                const double2 *__restrict__ taus) {
    __shared__ double2 pS[NB], qS[NB], Ws[NB], Vs[NB];
    __shared__ double red[8];
    __shared__ double2 ypart[4][TT];
    __shared__ double2 wsh;
    const int I = blockIdx.x, t = threadIdx.x;
    const double2 tj = taus[j];
    // p = V^H v, q = W^H v summed over row blocks
    if (t < 2 * c) {
        const bool isv = t < c;
        const int cc = isv ? t : t - c;
        double2 acc = cmk(0.0, 0.0);
        for (int b = 0; b < mt; ++b) acc = cadd(acc, pq[((int64_t)b * 2 + (isv ? 0 : 1)) * NB + cc]);
        if (isv) pS[cc] = acc; else qS[cc] = acc;
    }
    double part = 0.0;
    for (int b = t; b < nt; b += blockDim.x) part += tdot[b];
    const double vAv = block_sum(part, red);  // contains barriers: pS/qS visible after it
    double qp = 0.0;
    for (int cc = 0; cc < c; ++cc) qp += cmulc(qS[cc], pS[cc]).x;
    const double uv = vAv - 2.0 * qp;
    const double a2 = -0.5 * cabs2(tj) * uv;
    // y for rows of this block: slot sums split over 4 thread groups
    {
        const int r = t & 63, g = t >> 6;
        double2 acc = cmk(0.0, 0.0);
        for (int sl = g; sl < mt; sl += 4) acc = cadd(acc, P[((int64_t)I * mt + sl) * TT + r]);
        ypart[g][r] = acc;
    }
    // w at row s (first trailing row), needed by every block for column j+1
    if (next_in_panel && t == 0) {
        double2 y = cmk(0.0, 0.0);
        for (int sl = 0; sl < mt; ++sl) y = cadd(y, P[(int64_t)sl * TT + 0]);
        double2 u = y;
        for (int cc = 0; cc < c; ++cc) {
            u = csub(u, cmul(M[s + (int64_t)(p0 + cc) * lda], qS[cc]));
            u = csub(u, cmul(W[s + (int64_t)cc * lda], pS[cc]));
        }
        wsh = cadd(cmul(tj, u), cmk(a2, 0.0));  // v[s] = 1
    }
    if (next_in_panel && t < c) {
        Ws[t] = W[s + (int64_t)t * lda];
        Vs[t] = M[s + (int64_t)(p0 + t) * lda];
    }
    __syncthreads();
    if (t < TT) {
        const int row = s + I * TT + t;
        if (row < n) {
            const double2 y = cadd(cadd(ypart[0][t], ypart[1][t]), cadd(ypart[2][t], ypart[3][t]));
            double2 u = y;
            for (int cc = 0; cc < c; ++cc) {
                u = csub(u, cmul(M[row + (int64_t)(p0 + cc) * lda], qS[cc]));
                u = csub(u, cmul(W[row + (int64_t)cc * lda], pS[cc]));
            }
            const double2 v = vbuf[row];
            const double2 w = cfma(cmk(a2, 0.0), v, cmul(tj, u));
            W[row + (int64_t)c * lda] = w;
            if (next_in_panel) {
                // column j+1 of A_cur: subtract sum over panel columns 0..c of
                // V(row,cc) conj(W(s,cc)) + W(row,cc) conj(V(s,cc))
                double2 a = M[row + (int64_t)(j + 1) * lda];
                for (int cc = 0; cc < c; ++cc) {
                    a = csub(a, cmul(M[row + (int64_t)(p0 + cc) * lda], cconj(Ws[cc])));
                    a = csub(a, cmul(W[row + (int64_t)cc * lda], cconj(Vs[cc])));
                }
                a = csub(a, cmul(v, cconj(wsh)));
                a = csub(a, w);  // W(row,c) * conj(V(s,c)) with V(s,c) = v[s] = 1
                M[row + (int64_t)(j + 1) * lda] = a;
            }
        }
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

// T factor of the block reflector of panel b: H_p0 ... H_{p0+kb-1} = I - V T V^H
// (forward, columnwise):  T(i,i) = tau_i,  T(0:i, i) = -tau_i T(0:i,0:i) V(:,0:i)^H v_i.
__global__ void __launch_bounds__(256) tfactor_kernel(const double2 *__restrict__ M, int64_t lda, int n,
                                                      const double2 *__restrict__ taus, double2 *Tout) {
    __shared__ double2 Vc[64][NB + 1];
    __shared__ double2 G[NB][NB + 1];
    __shared__ double2 Ts[NB][NB + 1];
    const int b = blockIdx.x, t = threadIdx.x;
    const int p0 = b * NB;
    const int kb = min(NB, n - 1 - p0);
    // G = V^H V over rows p0+1..n-1, pairs (c1 <= c2)
    const int npair = kb * (kb + 1) / 2;
    double2 acc[3] = {cmk(0, 0), cmk(0, 0), cmk(0, 0)};
    int pc1[3], pc2[3];
    for (int k = 0; k < 3; ++k) {
        const int pidx = t + k * 256;
        int c1 = 0, rem = pidx;
        while (c1 < kb && rem >= kb - c1) { rem -= kb - c1; ++c1; }
        pc1[k] = c1; pc2[k] = c1 + rem;
    }
    for (int r0 = p0 + 1; r0 < n; r0 += 64) {
        for (int idx = t; idx < 64 * NB; idx += 256) {
            const int r = idx & 63, cc = idx >> 6;
            Vc[r][cc] = (r0 + r < n && cc < kb) ? M[(r0 + r) + (int64_t)(p0 + cc) * lda] : cmk(0.0, 0.0);
        }
        __syncthreads();
        for (int k = 0; k < 3; ++k) {
            if (t + k * 256 >= npair) break;
            const int c1 = pc1[k], c2 = pc2[k];
            for (int r = 0; r < 64; ++r) acc[k] = cfmac(Vc[r][c1], Vc[r][c2], acc[k]);
        }
        __syncthreads();
    }
    for (int k = 0; k < 3; ++k)
        if (t + k * 256 < npair) G[pc1[k]][pc2[k]] = acc[k];
    for (int idx = t; idx < NB * NB; idx += 256) Ts[idx % NB][idx / NB] = cmk(0.0, 0.0);
    __syncthreads();
    if (t == 0)
        for (int i = 0; i < kb; ++i) Ts[i][i] = taus[p0 + i];
    __syncthreads();
    for (int i = 1; i < kb; ++i) {
        // z = T(0:i,0:i) G(0:i, i); T(0:i, i) = -tau_i z
        double2 z = cmk(0.0, 0.0);
        if (t < i) {
            for (int l = t; l < i; ++l) z = cfma(Ts[t][l], G[l][i], z);
        }
        __syncthreads();
        if (t < i) Ts[t][i] = cscale(cmul(taus[p0 + i], z), -1.0);
        __syncthreads();
    }
    double2 *To = Tout + (int64_t)b * NB * NB;
    for (int idx = t; idx < NB * NB; idx += 256) To[idx] = Ts[idx % NB][idx / NB];
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
        for (int c = 0; c < kb; ++c) {
            const int j = p0 + c, s = j + 1, m = n - s;
            const int mt = (m + TT - 1) / TT, nt = mt * (mt + 1) / 2;
            hipLaunchKernelGGL(refl_kernel, dim3(1), dim3(512), 0, st, w.M, w.lda, n, j, w.vbuf, w.tau, w.d, w.e);
            hipLaunchKernelGGL(hemv_kernel, dim3(nt), dim3(256), 0, st, w.M, w.lda, n, s, mt, w.vbuf, w.W, p0, c,
                               w.P, w.tdot, w.pq);
            const int next_in_panel = (c + 1 < kb) ? 1 : 0;
            hipLaunchKernelGGL(w_kernel, dim3(mt), dim3(256), 0, st, w.M, w.lda, n, j, s, mt, nt, w.vbuf, w.W,
                               p0, c, next_in_panel, w.P, w.tdot, w.pq, w.tau);
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
    hipLaunchKernelGGL(refl_kernel, dim3(1), dim3(512), 0, st, w.M, w.lda, n, n - 1, w.vbuf, w.tau, w.d, w.e);
    return hipGetLastError();
}

hipError_t large_compute_T(const LargeWs &w, hipStream_t st) {
    dim3 grid((w.n + 255) / 256, w.n);
    hipLaunchKernelGGL(clean_kernel, grid, dim3(256), 0, st, w.M, w.lda, w.n);
    if (w.npanel > 0)
        hipLaunchKernelGGL(tfactor_kernel, dim3(w.npanel), dim3(256), 0, st, w.M, w.lda, w.n, w.tau, w.T);
    return hipGetLastError();
}

}  // namespace psd
