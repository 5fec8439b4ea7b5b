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
// Once the trailing matrix from a panel boundary has order <= LG_TAIL, one
// workgroup per block finishes the reduction in LDS (tail_kernel): the
// launches of those columns would cost far more than their work.
//
// Per column two launches: the tiled HEMV over the lower triangle (one
// workgroup per 64x64 tile; each first rebuilds the column's reflector from
// the sigma partials, identically), and the w/next-column step (one workgroup
// per 64 rows), which also extends the block-reflector factor T and leaves
// the next column's sigma partials.  Partial sums go to fixed slots, no
// atomics: the result is deterministic.  Only the lower triangle (row >=
// column) of M is ever read.
#include <algorithm>

#include "common.h"
#include "large.h"
#include "timing.h"

namespace psd {

namespace {

constexpr int TT = LG_TILE;
constexpr int NB = LG_NB;
constexpr int TAIL = LG_TAIL;
// per-wave register staging below: 2c < 4 * (NB / 2) panel columns, c*c <= NB*NB
// T-factor entries over 256 threads, TT / 4 tile columns per wave
static_assert(TT == 64 && NB % 8 == 0 && (NB * NB) % 256 == 0, "staging layout");

// svec -> lower triangle of M (M = conj X, see common.h); flags non-finite.
__global__ void __launch_bounds__(256) unpack_kernel(const double *__restrict__ x, double2 *M, int64_t lda, int n,
                                                     int *status, int64_t zs, const int64_t *__restrict__ ioff) {
    const int b = blockIdx.z;
    M = member_ptr(M, zs, b);
    status = member_ptr(status, zs, b);
    if (ioff) x += ioff[b];
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
__device__ void norm_body(const double2 *__restrict__ M, int64_t lda, int n, int j, double *npart) {
    __shared__ double red[16];
    const double2 *col = M + (int64_t)j * lda;
    double part = 0.0;
    for (int r = j + 2 + threadIdx.x; r < n; r += blockDim.x) part += cabs2(col[r]);
    // wave sums (every lane active), then the waves' in order
    part = wave_sum_dpp(part);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) sum += red[k];
        npart[0] = sum;
    }
}

__global__ void __launch_bounds__(512) norm_kernel(const double2 *__restrict__ M, int64_t lda, int n, int j,
                                                   double *npart, int64_t zs) {
    norm_body(member_ptr(M, zs, blockIdx.z), lda, n, j, member_ptr(npart, zs, blockIdx.z));
}

// Reflector of column j (recomputed identically by every workgroup from the
// sigma partials), then tile (I, J), J <= I, of the trailing matrix
// A = M[s:, s:] (s = j+1) times v:
//   direct part  A_IJ v_J      -> P[I][slot J]
//   adjoint part A_IJ^H v_I    -> P[J][slot I]     (I > J only)
//   tdot[tile]  = w * Re(v_I^H A_IJ v_J), w = 1 (diagonal) or 2
// The tile stays in registers (thread: row = lane, columns g + 4k): the row
// sums are per-thread partials over 16 columns summed over the 4 waves, the
// column sums a split butterfly over the 64 lanes of the wave that owns the
// column.  A diagonal tile holds its stored lower part L + D (D real), and
// H v = (L + D) v + L^H v: the direct part over the lower part, the adjoint
// part over the strict lower part added to the same rows.  Only the short
// vectors pass through LDS, so three workgroups fit on a CU.
// Diagonal-tile workgroups write v for their rows into vbuf.  The panel dot
// products p = V^H v and q = W^H v (c panel columns done) are summed per
// block row by workgroups of their own (hemv_pq), so that no workgroup of
// the launch waits on a second memory round trip.
struct HemvLds {
    double2 vI[TT], vJ[TT];
    double2 rowp[4][TT], colp[TT];
};

__device__ void hemv_tile(const double2 *__restrict__ M, int64_t lda, int n, int j, int mt,
                          const double *__restrict__ npart, int nparts, double2 *vbuf,
                          const double2 *__restrict__ W, int p0, int c, double2 *P, double *tdot, double2 *pq,
                          double2 *taus, double *d, double *e, int b, HemvLds &L) {
    auto &vI = L.vI;
    auto &vJ = L.vJ;
    auto &rowp = L.rowp;
    auto &colp = L.colp;
    const int s = j + 1;
    int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= b) ++I;
    while (I * (I + 1) / 2 > b) --I;
    const int J = b - I * (I + 1) / 2;
    const int t = threadIdx.x, lane = t & 63, g = t >> 6;
    const int r0 = s + I * TT, c0 = s + J * TT;
    const double2 *colj = M + (int64_t)j * lda;
    const bool diag = I == J;
    const bool rowok = r0 + lane < n;
    // every global load of the tile issued at once: one memory round trip
    // (a loop that sums loaded values waits for its loads before anything
    // after it is issued, so only the rare partials beyond 64 are looped over,
    // after the tile's loads)
    double sp = lane < nparts ? npart[lane] : 0.0;  // sigma: every wave sums the same partials in the same order
    const double2 alpha = colj[s];
    const double djj = (b == 0 && t == 0) ? colj[j].x : 0.0;
    // the column's entries for v before the tile: loads complete in order,
    // so the reflector and v are formed while the tile is still in flight
    const int vrow = (t < TT ? r0 : c0) + lane;  // threads < 2*TT: entries of v_I, v_J
    const double2 cv = (t < 2 * TT && vrow < n && vrow != s) ? colj[vrow] : cmk(0.0, 0.0);
    double2 tv[TT / 4];  // tile column g + 4k, row lane (diagonal tile: lower part only)
#pragma unroll
    for (int k = 0; k < TT / 4; ++k) {
        const int cc = g + 4 * k, col = c0 + cc;
        tv[k] = (rowok && col < n && (!diag || lane >= cc)) ? M[(r0 + lane) + (int64_t)col * lda] : cmk(0.0, 0.0);
    }
    for (int k = lane + 64; k < nparts; k += 64) sp += npart[k];
    const double sigma = wave_sum_dpp(sp);
    const Refl h = make_refl(alpha, sigma);
    if (t < 2 * TT) {
        double2 v = cmk(0.0, 0.0);
        if (vrow == s) v = cmk(1.0, 0.0);
        else if (vrow < n) v = cmul(cv, h.scale);
        if (t < TT) vI[t] = v; else vJ[t - TT] = v;
    }
    __syncthreads();
    if (b == 0 && t == 0) {
        d[j] = djj;
        e[j] = h.beta;
        taus[j] = h.tau;
    }
    // direct part: this thread's row over its 16 columns; adjoint part: the
    // 16 column terms of this row, summed over the lanes below
    const double2 vl = vI[lane];
    double2 racc = cmk(0.0, 0.0);
    double pv[TT / 2];  // {re, im} of column g + 4k at 2k, 2k + 1
#pragma unroll
    for (int k = 0; k < TT / 4; ++k) {
        const int cc = g + 4 * k;
        double2 a = tv[k];
        if (diag && lane == cc) a.y = 0.0;  // the diagonal is real
        racc = cfma(a, vJ[cc], racc);
        const double2 z = (diag && lane == cc) ? cmk(0.0, 0.0) : cmulc(tv[k], vl);  // conj(A) v_I
        pv[2 * k] = z.x;
        pv[2 * k + 1] = z.y;
    }
    rowp[g][lane] = racc;
    {
        const double sum = wave_sum_split(pv);  // lane l: value l / 2
        if ((lane & 1) == 0) reinterpret_cast<double *>(&colp[g + 4 * (lane >> 2)])[(lane >> 1) & 1] = sum;
    }
    __syncthreads();
    if (t < TT) {
        double2 y = cadd(cadd(rowp[0][t], rowp[1][t]), cadd(rowp[2][t], rowp[3][t]));
        if (diag) y = cadd(y, colp[t]);
        P[((int64_t)I * mt + J) * TT + t] = y;
        if (diag && r0 + t < n) vbuf[r0 + t] = vI[t];
        const double dv = wave_sum_dpp(cmulc(vI[t], y).x);  // wave 0, every lane
        if (t == 0) tdot[b] = diag ? dv : 2.0 * dv;
    } else if (t < 2 * TT && !diag) {
        const int cc = t - TT;
        P[((int64_t)J * mt + I) * TT + cc] = colp[cc];
    }
    __syncthreads();  // LDS reuse by a following call in the same workgroup
}

// p = V^H v and q = W^H v over the 64 rows of block row I (2c columns,
// column q on wave q % 4 with the rows on the lanes): the reflector is
// rebuilt from the sigma partials as by the tiles, and every load is issued
// at once.
__device__ void hemv_pq(const double2 *__restrict__ M, int64_t lda, int n, int j, const double *__restrict__ npart,
                        int nparts, const double2 *__restrict__ W, int p0, int c, double2 *pq, int I) {
    const int s = j + 1;
    const int t = threadIdx.x, lane = t & 63, g = t >> 6;
    const int r0 = s + I * TT;
    const int row = r0 + lane;
    const bool rowok = row < n;
    const double2 *colj = M + (int64_t)j * lda;
    double sp = lane < nparts ? npart[lane] : 0.0;  // as in hemv_tile
    const double2 alpha = colj[s];
    const double2 cv = (rowok && row != s) ? colj[row] : cmk(0.0, 0.0);
    double2 xq[TT / 4];
#pragma unroll
    for (int k = 0; k < TT / 4; ++k) {
        const int q = g + 4 * k;
        xq[k] = cmk(0.0, 0.0);
        if (q < 2 * c && rowok) {
            const double2 *col = (q < c) ? (M + (int64_t)(p0 + q) * lda) : (W + (int64_t)(q - c) * lda);
            xq[k] = col[row];
        }
    }
    for (int k = lane + 64; k < nparts; k += 64) sp += npart[k];
    const double sigma = wave_sum_dpp(sp);
    const Refl h = make_refl(alpha, sigma);
    double2 vl = cmk(0.0, 0.0);
    if (row == s) vl = cmk(1.0, 0.0);
    else if (rowok) vl = cmul(cv, h.scale);
    double pw[TT / 2];  // {re, im} of column g + 4k at 2k, 2k + 1
#pragma unroll
    for (int k = 0; k < TT / 4; ++k) {
        const double2 pr = cmulc(xq[k], vl);
        pw[2 * k] = pr.x;
        pw[2 * k + 1] = pr.y;
    }
    const double sum = wave_sum_split(pw);  // lane l: value l / 2
    const int q = g + 4 * (lane >> 2);
    if ((lane & 1) == 0 && q < 2 * c)
        reinterpret_cast<double *>(pq)[2 * (((int64_t)I * 2 + (q < c ? 0 : 1)) * NB + (q < c ? q : q - c)) +
                                       ((lane >> 1) & 1)] = sum;
}

// Workgroups 0 .. nt-1: the tiles; nt .. nt+mt-1 (when c > 0): the panel dot
// products of block row blockIdx.x - nt.
__global__ void __launch_bounds__(256, 3) hemv_kernel(const double2 *__restrict__ M, int64_t lda, int n, int j,
                                                   int mt, const double *__restrict__ npart, int nparts,
                                                   double2 *vbuf, const double2 *__restrict__ W, int p0, int c,
                                                   double2 *P, double *tdot, double2 *pq, double2 *taus,
                                                   double *d, double *e, int64_t zs) {
    __shared__ HemvLds L;
    const int b = blockIdx.z;
    M = member_ptr(M, zs, b);
    npart = member_ptr(npart, zs, b);
    vbuf = member_ptr(vbuf, zs, b);
    W = member_ptr(W, zs, b);
    P = member_ptr(P, zs, b);
    tdot = member_ptr(tdot, zs, b);
    pq = member_ptr(pq, zs, b);
    taus = member_ptr(taus, zs, b);
    d = member_ptr(d, zs, b);
    e = member_ptr(e, zs, b);
    const int nt = mt * (mt + 1) / 2;
    if ((int)blockIdx.x >= nt) {
        hemv_pq(M, lda, n, j, npart, nparts, W, p0, c, pq, (int)blockIdx.x - nt);
        return;
    }
    hemv_tile(M, lda, n, j, mt, npart, nparts, vbuf, W, p0, c, P, tdot, pq, taus, d, e, blockIdx.x, L);
}

struct WLds {
    double2 pS[NB], qS[NB], Ws[NB], Vs[NB];
    double2 Tl[NB][NB + 1];
    double red[8];
    double2 ypart[4][TT], upart[4][TT], apart[4][TT];
    double2 wsh;
};

// Rows of block I (64 rows from s): stores v into the reflector column j,
// w = tau u + a2 v into W[:, c] with u = y - V q - W p, and -- when column
// j+1 belongs to the same panel -- applies the panel update to column j+1 and
// writes its sigma partial (rows > j+2).  Workgroup 0 also appends column c
// of the block-reflector factor: T(c,c) = tau, T(0:c,c) = -tau T(0:c,0:c) p,
// since p = V^H v_c = G(0:c, c) for v_c vanishing above row j+1.
__device__ void w_rows(double2 *M, int64_t lda, int n, int j, int mt, int nt, const double2 *__restrict__ vbuf,
                       double2 *W, int p0, int c, int next_in_panel, const double2 *__restrict__ P,
                       const double *__restrict__ tdot, const double2 *__restrict__ pq,
                       const double2 *__restrict__ taus, double2 *Tb, double *npart, int I, WLds &L) {
    auto &pS = L.pS;
    auto &qS = L.qS;
    auto &Ws = L.Ws;
    auto &Vs = L.Vs;
    auto &Tl = L.Tl;
    auto &red = L.red;
    auto &ypart = L.ypart;
    auto &upart = L.upart;
    auto &apart = L.apart;
    auto &wsh = L.wsh;
    const int s = j + 1;
    const int t = threadIdx.x;
    const int r = t & 63, g = t >> 6;
    const int row = s + I * TT + r;
    const bool rowok = row < n;
    // Every global load is issued here, ahead of its use (the stores below
    // could alias them, so the compiler would not hoist them): one memory
    // round trip.  A loop that sums loaded values waits for its loads before
    // anything after it is issued, so the first chunk of each sum is loaded
    // here and only the chunks beyond it (n > 4096) are looped over, after
    // every first load.  At most mt <= 64 workgroups run, so the registers
    // this takes cost no occupancy.
    const double2 tj = taus[j];
    double2 pqv[NB / 2];  // p (q < c) / q (q >= c) partials of column q = g + 4k, row blocks on the lanes
#pragma unroll
    for (int k = 0; k < NB / 2; ++k) {
        const int q = g + 4 * k;
        const double2 *src = pq + (q < c ? q : NB + q - c);  // row block bb at src[bb * 2 * NB]
        pqv[k] = (q < 2 * c && r < mt) ? src[(int64_t)r * 2 * NB] : cmk(0.0, 0.0);
    }
    double2 wsv = cmk(0.0, 0.0), vsv = cmk(0.0, 0.0);
    if (next_in_panel && t >= 64 && t < 64 + c) {
        wsv = W[s + (int64_t)(t - 64) * lda];
        vsv = M[s + (int64_t)(p0 + t - 64) * lda];
    }
    double2 tlv[NB * NB / 256];
#pragma unroll
    for (int k = 0; k < NB * NB / 256; ++k) {
        const int idx = t + 256 * k;
        tlv[k] = (I == 0 && idx < c * c) ? Tb[(idx % c) + (idx / c) * NB] : cmk(0.0, 0.0);
    }
    // tile terms v_I^H A v_J (256 threads, chunks of 8 x 256) and the
    // partials of y = A v for this row (4 groups, chunks of 16 x 4)
    double tv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) tv[u] = (t + 256 * u < nt) ? tdot[t + 256 * u] : 0.0;
    double2 yv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u)
        yv[u] = (g + 4 * u < mt) ? P[((int64_t)I * mt + g + 4 * u) * TT + r] : cmk(0.0, 0.0);
    double2 vr[NB / 4], wr[NB / 4];  // panel columns g + 4k of V and W at this row
#pragma unroll
    for (int k = 0; k < NB / 4; ++k) {
        const int cc = g + 4 * k;
        const bool ok = rowok && cc < c;
        vr[k] = ok ? M[row + (int64_t)(p0 + cc) * lda] : cmk(0.0, 0.0);
        wr[k] = ok ? W[row + (int64_t)cc * lda] : cmk(0.0, 0.0);
    }
    double2 ys = (next_in_panel && g == 0 && r < mt) ? P[(int64_t)r * TT] : cmk(0.0, 0.0);
    double2 vrow = cmk(0.0, 0.0), mnext = cmk(0.0, 0.0);
    if (t < TT && rowok) {
        vrow = vbuf[row];
        if (next_in_panel) mnext = M[row + (int64_t)(j + 1) * lda];
    }
    // the chunks beyond the first (n > 4096), after every first load
#pragma unroll
    for (int k = 0; k < NB / 2; ++k) {
        const int q = g + 4 * k;
        const double2 *src = pq + (q < c ? q : NB + q - c);
        if (q < 2 * c)
            for (int bb = r + 64; bb < mt; bb += 64) pqv[k] = cadd(pqv[k], src[(int64_t)bb * 2 * NB]);
    }
    // (sums start from their first term: an added constant zero would be
    // moved into the predicated load and wait for it there)
    double part = tv[0];
#pragma unroll
    for (int u = 1; u < 8; ++u) part += tv[u];
    for (int base = t + 8 * 256; base < nt; base += 8 * 256) {
#pragma unroll
        for (int u = 0; u < 8; ++u) tv[u] = (base + 256 * u < nt) ? tdot[base + 256 * u] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) part += tv[u];
    }
    double2 y = yv[0];
#pragma unroll
    for (int u = 1; u < 16; ++u) y = cadd(y, yv[u]);
    for (int base = g + 64; base < mt; base += 64) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
            yv[u] = (base + 4 * u < mt) ? P[((int64_t)I * mt + base + 4 * u) * TT + r] : cmk(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < 16; ++u) y = cadd(y, yv[u]);
    }
    if (next_in_panel && g == 0)
        for (int sl = r + 64; sl < mt; sl += 64) ys = cadd(ys, P[(int64_t)sl * TT]);
    // p = V^H v, q = W^H v
    {
        double pv[NB];  // {re, im} of column g + 4k at 2k, 2k + 1
#pragma unroll
        for (int k = 0; k < NB / 2; ++k) {
            pv[2 * k] = pqv[k].x;
            pv[2 * k + 1] = pqv[k].y;
        }
        const double sum = wave_sum_split(pv);  // lane l: value l / 2
        const int q = g + 4 * (r >> 2);
        if ((r & 1) == 0 && q < 2 * c)
            (q < c ? reinterpret_cast<double *>(pS) + 2 * q : reinterpret_cast<double *>(qS) + 2 * (q - c))[(r >> 1) & 1] =
                sum;
    }
    if (next_in_panel && t >= 64 && t < 64 + c) {
        Ws[t - 64] = wsv;
        Vs[t - 64] = vsv;
    }
#pragma unroll
    for (int k = 0; k < NB * NB / 256; ++k) {
        const int idx = t + 256 * k;
        if (I == 0 && idx < c * c) Tl[idx % c][idx / c] = tlv[k];
    }
    // v^H A v: per-wave sums, then the four in order (the barrier also makes
    // pS/qS/Ws/Vs/Tl visible)
    part = wave_sum_dpp(part);
    if (r == 0) red[g] = part;
    __syncthreads();
    double vAv = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) vAv += red[k];
    // Re q^H p: lanes over the panel columns (every wave, same order)
    const double qp = wave_sum_dpp(r < c ? cmulc(qS[r], pS[r]).x : 0.0);
    const double a2 = -0.5 * cabs2(tj) * (vAv - 2.0 * qp);
    // block-reflector factor, column c: row i on the 8 lanes 8i..8i+7
    if (I == 0) {
        const int ti = t >> 3, ch = t & 7;
        double2 z = cmk(0.0, 0.0);
        if (ti < c)
            for (int l = ti + ch; l < c; l += 8) z = cfma(Tl[ti][l], pS[l], z);
        // sum over the 8 lanes of row ti (every lane of the workgroup active)
        z = cadd(z, cmk(xor_lane<1>(z.x, t & 63), xor_lane<1>(z.y, t & 63)));
        z = cadd(z, cmk(xor_lane<2>(z.x, t & 63), xor_lane<2>(z.y, t & 63)));
        z = cadd(z, cmk(xor_lane<4>(z.x, t & 63), xor_lane<4>(z.y, t & 63)));
        if (ch == 0 && ti <= c) Tb[ti + c * NB] = (ti == c) ? tj : cscale(cmul(tj, z), -1.0);
    }
    // V q + W p and (for column j+1) the panel terms, split over 4 groups
    {
        double2 u = cmk(0.0, 0.0), a = cmk(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < NB / 4; ++k) {
            const int cc = g + 4 * k;
            if (cc < c) {
                u = cfma(vr[k], qS[cc], u);
                u = cfma(wr[k], pS[cc], u);
                if (next_in_panel) {
                    a = cfma(vr[k], cconj(Ws[cc]), a);
                    a = cfma(wr[k], cconj(Vs[cc]), a);
                }
            }
        }
        ypart[g][r] = y;
        upart[g][r] = u;
        apart[g][r] = a;
    }
    // w at row s, needed by every block for column j+1 (wave 0)
    if (next_in_panel && g == 0) {
        // y(s) - (V q)(s) - (W p)(s), the panel columns on the lanes
        if (r < c) ys = csub(ys, cadd(cmul(Vs[r], qS[r]), cmul(Ws[r], pS[r])));
        double yv[2] = {ys.x, ys.y};
        const double ysum = wave_sum_split(yv);  // lanes 0..31: re, 32..63: im
        const double2 yt = cmk(readlane_double(ysum, 0), readlane_double(ysum, 32));
        if (r == 0) wsh = cadd(cmul(tj, yt), cmk(a2, 0.0));  // v[s] = 1
    }
    __syncthreads();
    double nrm = 0.0;
    if (t < TT && rowok) {
        const double2 yy = cadd(cadd(ypart[0][r], ypart[1][r]), cadd(ypart[2][r], ypart[3][r]));
        const double2 vq = cadd(cadd(upart[0][r], upart[1][r]), cadd(upart[2][r], upart[3][r]));
        const double2 v = vrow;
        M[row + (int64_t)j * lda] = v;
        const double2 w = cfma(cmk(a2, 0.0), v, cmul(tj, csub(yy, vq)));
        W[row + (int64_t)c * lda] = w;
        if (next_in_panel) {
            // column j+1 of A_cur = A - V W^H - W V^H over panel columns 0..c
            const double2 pa = cadd(cadd(apart[0][r], apart[1][r]), cadd(apart[2][r], apart[3][r]));
            double2 a = csub(mnext, pa);
            a = csub(a, cmul(v, cconj(wsh)));
            a = csub(a, w);  // W(row,c) conj(V(s,c)), V(s,c) = 1
            M[row + (int64_t)(j + 1) * lda] = a;
            if (row > j + 2) nrm = cabs2(a);
        }
    }
    // sigma partial of column j+1 over these rows: only wave 0 holds rows
    if (next_in_panel && g == 0) {
        const double sum = wave_sum_dpp(nrm);
        if (t == 0) npart[I] = sum;
    }
}

__global__ void __launch_bounds__(256) w_kernel(double2 *M, int64_t lda, int n, int j, int mt, int nt,
                                                const double2 *__restrict__ vbuf, double2 *W, int p0, int c,
                                                int next_in_panel, const double2 *__restrict__ P,
                                                const double *__restrict__ tdot, const double2 *__restrict__ pq,
                                                const double2 *__restrict__ taus, double2 *Tb, double *npart,
                                                int64_t zs) {
    __shared__ WLds L;
    const int b = blockIdx.z;
    M = member_ptr(M, zs, b);
    vbuf = member_ptr(vbuf, zs, b);
    W = member_ptr(W, zs, b);
    P = member_ptr(P, zs, b);
    tdot = member_ptr(tdot, zs, b);
    pq = member_ptr(pq, zs, b);
    taus = member_ptr(taus, zs, b);
    Tb = member_ptr(Tb, zs, b);
    npart = member_ptr(npart, zs, b);
    w_rows(M, lda, n, j, mt, nt, vbuf, W, p0, c, next_in_panel, P, tdot, pq, taus, Tb, npart, blockIdx.x, L);
}

// The last columns in one workgroup.  The lower triangle of the trailing
// matrix A = M[p0:, p0:] (order m0 = n - p0 <= TAIL; every earlier panel is
// already applied) is held in LDS packed by rows, and the unblocked steps of
// the same reduction run there, column k after column k-1:
//   v from column k (make_refl), y = A22 v, w = tau y - 1/2 |tau|^2 (v^H y) v,
//   A22 -= v w^H + w v^H
// (the panel formulas with no earlier panel columns), each v overwriting the
// column it came from.  Then the block-reflector factor of every panel of the
// tail follows from the Gram matrix G = V^H V of its reflectors:
//   T(c, c) = tau_c,  T(0:c, c) = -tau_c T(0:c, 0:c) G(0:c, c),
// the recurrence the per-column step applies with p = V^H v_c = G(0:c, c).
// One workgroup of 1024 threads per block (grid z: group member).
struct TailLds {
    double2 A[TAIL * (TAIL + 1) / 2];  // row i at i(i+1)/2, columns 0..i
    double2 v[TAIL], w[TAIL];           // w: y = A22 v of the current column
    double2 tau[TAIL];
    double2 G[NB * NB], Tf[NB * NB];    // column-major, leading dimension NB
};

__device__ __forceinline__ int tpk(int i, int l) { return i * (i + 1) / 2 + l; }

__global__ void __launch_bounds__(1024) tail_kernel(double2 *M, int64_t lda, int n, int p0, double2 *taus,
                                                    double *d, double *e, double2 *T, int64_t zs) {
    __shared__ TailLds L;
    const int b = blockIdx.z;
    M = member_ptr(M, zs, b);
    taus = member_ptr(taus, zs, b);
    d = member_ptr(d, zs, b);
    e = member_ptr(e, zs, b);
    T = member_ptr(T, zs, b);
    const int m0 = n - p0;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int ri = t >> 3, sub = t & 7;  // phases over rows: 8 threads per row
    // lower triangle of A, column-major in HBM: all loads issued, then stored
    {
        constexpr int CH = (TAIL * TAIL + 1023) / 1024;
        double2 buf[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int idx = t + 1024 * u, l = idx / m0, i = idx - l * m0;
            buf[u] = (idx < m0 * m0 && i >= l) ? M[(p0 + i) + (int64_t)(p0 + l) * lda] : cmk(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int idx = t + 1024 * u, l = idx / m0, i = idx - l * m0;
            if (idx < m0 * m0 && i >= l) L.A[tpk(i, l)] = buf[u];
        }
    }
    __syncthreads();
    for (int k = 0; k < m0 - 1; ++k) {
        const int k1 = k + 1;
        // reflector of column k and v (wave 0)
        if (wv == 0) {
            double sp = 0.0;
            for (int r = k + 2 + lane; r < m0; r += 64) sp += cabs2(L.A[tpk(r, k)]);
            const double sigma = wave_sum_dpp(sp);
            const Refl h = make_refl(L.A[tpk(k1, k)], sigma);
            for (int r = k1 + lane; r < m0; r += 64) {
                const double2 vr = (r == k1) ? cmk(1.0, 0.0) : cmul(L.A[tpk(r, k)], h.scale);
                L.v[r] = vr;
                L.A[tpk(r, k)] = vr;
            }
            if (lane == 0) {
                L.tau[k] = h.tau;
                d[p0 + k] = L.A[tpk(k, k)].x;
                e[p0 + k] = h.beta;
                taus[p0 + k] = h.tau;
            }
        }
        __syncthreads();
        // y = A22 v: row i over columns k1 + sub + 8q (the diagonal is real),
        // eight loads issued per chunk before they are used
        {
            const int i = k1 + ri;
            double2 acc = cmk(0.0, 0.0);
            if (i < m0) {
                const int rowb = tpk(i, 0);
                for (int l0 = k1 + sub; l0 < m0; l0 += 64) {
                    double2 av[8], vv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int l = l0 + 8 * u;
                        av[u] = cmk(0.0, 0.0);
                        vv[u] = cmk(0.0, 0.0);
                        if (l < m0) {
                            vv[u] = L.v[l];
                            if (l < i) av[u] = L.A[rowb + l];
                            else if (l == i) av[u] = cmk(L.A[rowb + l].x, 0.0);
                            else av[u] = cconj(L.A[tpk(l, i)]);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc = cfma(av[u], vv[u], acc);
                }
            }
            acc = cadd(acc, cmk(xor_lane<1>(acc.x, lane), xor_lane<1>(acc.y, lane)));
            acc = cadd(acc, cmk(xor_lane<2>(acc.x, lane), xor_lane<2>(acc.y, lane)));
            acc = cadd(acc, cmk(xor_lane<4>(acc.x, lane), xor_lane<4>(acc.y, lane)));
            if (sub == 0 && i < m0) L.w[i] = acc;
        }
        __syncthreads();
        // a2 = -1/2 |tau|^2 v^H A v (every wave, the same sum), then
        // A22 -= v w^H + w v^H over the lower triangle with w = tau y + a2 v
        // formed where it is needed
        {
            double pv = 0.0;
            for (int r = k1 + lane; r < m0; r += 64) pv += cmulc(L.v[r], L.w[r]).x;
            const double vAv = wave_sum_dpp(pv);
            const double2 tk = L.tau[k];
            const double2 a2 = cmk(-0.5 * cabs2(tk) * vAv, 0.0);
            const int i = k1 + ri;
            if (i < m0) {
                const double2 vi = L.v[i], wi = cfma(a2, vi, cmul(tk, L.w[i]));
                const int rowb = tpk(i, 0);
                for (int l0 = k1 + sub; l0 <= i; l0 += 32) {
                    double2 av[4], vv[4], yy[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int l = l0 + 8 * u;
                        av[u] = vv[u] = yy[u] = cmk(0.0, 0.0);
                        if (l <= i) {
                            av[u] = L.A[rowb + l];
                            vv[u] = L.v[l];
                            yy[u] = L.w[l];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int l = l0 + 8 * u;
                        const double2 wl = cfma(a2, vv[u], cmul(tk, yy[u]));
                        if (l <= i) L.A[rowb + l] = csub(av[u], cadd(cmul(vi, cconj(wl)), cmul(wi, cconj(vv[u]))));
                    }
                }
            }
        }
        __syncthreads();
    }
    if (t == 0) d[n - 1] = L.A[tpk(m0 - 1, m0 - 1)].x;
    // reflectors to M (column p0 + k, rows below the diagonal)
    for (int idx = t; idx < m0 * m0; idx += 1024) {
        const int k = idx / m0, r = idx - k * m0;
        if (r > k && k < m0 - 1) M[(p0 + r) + (int64_t)(p0 + k) * lda] = L.A[tpk(r, k)];
    }
    // block-reflector factors of the tail's panels
    for (int pp = p0; pp < n - 1; pp += NB) {
        const int kb = min(NB, n - 1 - pp), kc0 = pp - p0;
        {
            const int a = t % NB, c = t / NB;  // NB * NB == 1024 pairs: one each
            if (c < kb && a < c) {
                double2 g = cmk(0.0, 0.0);
                for (int r = kc0 + c + 1; r < m0; ++r) g = cfma(cconj(L.A[tpk(r, kc0 + a)]), L.A[tpk(r, kc0 + c)], g);
                L.G[a + c * NB] = g;
            }
        }
        __syncthreads();
        // row a of T on lane a of wave 0, column by column (each entry needs
        // only the same row's earlier entries)
        if (wv == 0 && lane < kb) {
            const int a = lane;
            for (int c = a; c < kb; ++c) {
                double2 z = cmk(0.0, 0.0);
                for (int l = a; l < c; ++l) z = cfma(L.Tf[a + l * NB], L.G[l + c * NB], z);
                const double2 tc = L.tau[kc0 + c];
                const double2 val = (c == a) ? tc : cscale(cmul(tc, z), -1.0);
                L.Tf[a + c * NB] = val;
                T[(int64_t)(pp / NB) * NB * NB + a + c * NB] = val;
            }
        }
        __syncthreads();  // G and Tf reuse by the next panel
    }
}

// Zero the upper triangle (incl. diagonal) of the reflector columns so that
// column j of M is exactly v_j (v_j(j+1) = 1 is already stored).
__global__ void __launch_bounds__(256) clean_kernel(double2 *M, int64_t lda, int n, int64_t zs) {
    M = member_ptr(M, zs, blockIdx.z);
    const int j = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i > j || j >= n) return;
    M[i + (int64_t)j * lda] = cmk(0.0, 0.0);
}


}  // namespace

hipError_t large_unpack(const LargeWs &w, const double *x, hipStream_t st) {
    dim3 grid((w.n + 255) / 256, w.n, w.nmem);
    hipLaunchKernelGGL(unpack_kernel, grid, dim3(256), 0, st, x, w.M, w.lda, w.n, w.ksel, w.zs, w.ioff);
    return hipGetLastError();
}

hipError_t large_tridiag(const LargeWs &w, hipStream_t st) {
    const int n = w.n;
    // panels up to ptail by the per-column launches; from ptail (the first
    // panel boundary with n - ptail <= TAIL) one workgroup finishes in LDS
    const int ptail = n <= TAIL ? 0 : (n - TAIL + NB - 1) / NB * NB;
    for (int p0 = 0; p0 < ptail; p0 += NB) {
        const int kb = min(NB, n - 1 - p0);
        double2 *Tb = w.T + (int64_t)(p0 / NB) * NB * NB;
        hipLaunchKernelGGL(norm_kernel, dim3(1, 1, w.nmem), dim3(512), 0, st, w.M, w.lda, n, p0, w.npart, w.zs);
        int nparts = 1;
        for (int c = 0; c < kb; ++c) {
            const int j = p0 + c, m = n - j - 1;
            const int mt = (m + TT - 1) / TT, nt = mt * (mt + 1) / 2;
            const int slot = timing_begin(KF_HEMV, st);
            hipLaunchKernelGGL(hemv_kernel, dim3(nt + (c > 0 ? mt : 0), 1, w.nmem), dim3(256), 0, st, w.M, w.lda, n, j, mt, w.npart,
                               nparts, w.vbuf, w.W, p0, c, w.P, w.tdot, w.pq, w.tau, w.d, w.e, w.zs);
            timing_end(slot, st, 8.0 * (double)m * (double)(m + 1) * w.nmem);
            const int next_in_panel = (c + 1 < kb) ? 1 : 0;
            const int wslot = timing_begin(KF_WSTEP, st);
            hipLaunchKernelGGL(w_kernel, dim3(mt, 1, w.nmem), dim3(256), 0, st, w.M, w.lda, n, j, mt, nt, w.vbuf,
                               w.W, p0, c, next_in_panel, w.P, w.tdot, w.pq, w.tau, Tb, w.npart, w.zs);
            timing_end(wslot, st, 0.0);
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
            g.nmem = w.nmem;
            g.zs = w.zs;
            hipError_t e = gemm_launch(g, true, EPI_STORE, st);
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL(tail_kernel, dim3(1, 1, w.nmem), dim3(1024), 0, st, w.M, w.lda, n, ptail, w.tau, w.d, w.e,
                       w.T, w.zs);
    return hipGetLastError();
}

hipError_t large_compute_T(const LargeWs &w, hipStream_t st) {
    dim3 grid((w.n + 255) / 256, w.n, w.nmem);
    hipLaunchKernelGGL(clean_kernel, grid, dim3(256), 0, st, w.M, w.lda, w.n, w.zs);
    return hipGetLastError();
}

}  // namespace psd
