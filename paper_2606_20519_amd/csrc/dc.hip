// Divide-and-conquer eigensolver for the real symmetric tridiagonal T
// (Cuppen's method with the Gu-Eisenstat eigenvector formula), bottom-up:
//
//  * T is cut into nl = 2^L leaves of <= DC_LEAF rows.  At every cut
//    between rows m-1 and m, T = diag(T1, T2) + |beta| u u^T with
//    beta = e[m-1], u = e_{m-1} + sgn(beta) e_m, T1/T2 having their touching
//    diagonal entries reduced by |beta|.
//  * Leaves: implicit QL in LDS (one workgroup each).
//  * Merge of two solved halves (D1, Q1), (D2, Q2):
//      T = diag(Q1,Q2) (D + rho z z^T) diag(Q1,Q2)^T,
//      z = [last row of Q1, sgn(beta) first row of Q2] / sqrt2, rho = 2|beta|.
//    Deflation: components with rho|z_i| <= tol are eigenpairs already; two
//    close poles are combined by a plane rotation that zeroes one z entry.
//    The k remaining roots of 1 + rho sum z_i^2/(d_i - lambda) = 0 are found
//    one per thread in shifted coordinates lambda = d_o + tau (o the nearer
//    pole) by a safeguarded two-pole rational iteration; z is then recomputed
//    from the roots (Loewner), which makes the computed vectors
//    u_j = (zhat_i / (d_i - lambda_j))_i numerically orthogonal.
//    Q_new = diag(Q1, Q2) U is two FP64 MFMA GEMMs per merge, batched over
//    the merges of a level.
#include <algorithm>
#include <utility>

#include "common.h"
#include "large.h"
#include "ql.h"

namespace psd {

namespace {

constexpr double EPS = 2.220446049250313e-16;
constexpr int LEAF_MAX = 64;
constexpr int PREP_LDS_MAX = 6144;  // 20 bytes per element in LDS

__host__ __device__ inline int leaf_bound(int i, int n, int nl) { return (int)(((int64_t)i * n) / nl); }

// Vectors of the merge workspace (offsets in units of n; a merge [a,b) uses
// indices a..b-1 of each).
enum { DZ = 0, DDM, DDD, DDH, DZH, DTAU, DLAM, DZHAT, DRC, DRS, DRHO, DNRM, DCOUNT };
enum { IPERM = 0, IKEEP, IDEFL, IRP, IRN, IORG, ICOL, IROWK, ICOUNT };
enum { SK = 0, SND, SNR, SCOUNT };

__global__ void __launch_bounds__(256) dc_leaf_kernel(const double *__restrict__ d, const double *__restrict__ e,
                                                      int n, int nl, double *D, double *Q, int64_t ldq,
                                                      int *status, int64_t zs) {
    {
        const int mb = blockIdx.z;
        d = member_ptr(d, zs, mb);
        e = member_ptr(e, zs, mb);
        D = member_ptr(D, zs, mb);
        Q = member_ptr(Q, zs, mb);
        status = member_ptr(status, zs, mb);
    }
    __shared__ double dl[LEAF_MAX], el[LEAF_MAX], Z[LEAF_MAX * LEAF_MAX];
    __shared__ double rc[LEAF_MAX], rs[LEAF_MAX];
    __shared__ int ri[LEAF_MAX], rankv[LEAF_MAX];
    __shared__ int nrot_s, done_s;
    const int q = blockIdx.x, t = threadIdx.x;
    const int a = leaf_bound(q, n, nl), b = leaf_bound(q + 1, n, nl), sz = b - a;
    // A block whose input held a NaN or an infinity is solved as the zero
    // matrix (its output is overwritten with NaN at the end): every index the
    // merges derive from the data then stays well defined.
    const bool flagged = status[2] == ST_ENONFINITE;
    if (t < sz) {
        double dv = flagged ? 0.0 : d[a + t];
        if (!flagged && t == 0 && a > 0) dv -= fabs(e[a - 1]);
        if (!flagged && t == sz - 1 && b < n) dv -= fabs(e[b - 1]);
        dl[t] = dv;
        el[t] = (!flagged && t < sz - 1) ? e[a + t] : 0.0;
    }
    for (int idx = t; idx < sz * sz; idx += blockDim.x) Z[idx] = (idx % sz == idx / sz) ? 1.0 : 0.0;
    __syncthreads();
    const int st = ql_implicit(dl, el, Z, sz, sz, rc, rs, ri, &nrot_s, &done_s);
    if (t == 0 && st != ST_OK && status[2] == ST_OK) status[2] = st;
    if (t < sz) {
        const double v = dl[t];
        int rank = 0;
        for (int k = 0; k < sz; ++k) rank += (dl[k] < v) || (dl[k] == v && k < t);
        rankv[t] = rank;
    }
    __syncthreads();
    // Ranks are a permutation only if every value compares (no NaN, which a
    // finite input can still produce by overflow): otherwise keep the order.
    __shared__ int perm_ok;
    if (t == 0) {
        unsigned long long bits = 0;  // sz <= LEAF_MAX = 64 rows
        for (int k = 0; k < sz; ++k) bits |= 1ull << rankv[k];
        const bool perm = (sz == 64) ? (bits == ~0ull) : (bits == ((1ull << sz) - 1));
        perm_ok = perm ? 1 : 0;
        if (!perm && status[2] == ST_OK) status[2] = ST_ENONFINITE;
    }
    __syncthreads();
    if (t < sz) {
        if (!perm_ok) rankv[t] = t;
        D[a + rankv[t]] = dl[t];
    }
    __syncthreads();
    for (int idx = t; idx < sz * sz; idx += blockDim.x) {
        const int r = idx % sz, c = idx / sz;
        Q[(a + r) + (int64_t)(a + rankv[c]) * ldq] = Z[r + c * sz];
    }
}

struct MergeGeo {
    int a, m, b;
};
__device__ inline MergeGeo merge_geo(int level, int q, int n, int nl) {
    MergeGeo g;
    g.a = leaf_bound(q << level, n, nl);
    g.m = leaf_bound((q << level) + (1 << (level - 1)), n, nl);
    g.b = leaf_bound((q + 1) << level, n, nl);
    return g;
}

__global__ void __launch_bounds__(256) dc_prep_kernel(int level, int n, int nl, const double *__restrict__ e,
                                                      const double *__restrict__ Dcur, const double *Qcur,
                                                      double *Qnext, int64_t ldq, double *U, double *dv,
                                                      int *iv, int *sv, GemmDesc *gd, int use_lds, int *status,
                                                      int64_t zs) {
    {
        const int mb = blockIdx.z;
        status = member_ptr(status, zs, mb);
        e = member_ptr(e, zs, mb);
        Dcur = member_ptr(Dcur, zs, mb);
        Qcur = member_ptr(Qcur, zs, mb);
        Qnext = member_ptr(Qnext, zs, mb);
        U = member_ptr(U, zs, mb);
        dv = member_ptr(dv, zs, mb);
        iv = member_ptr(iv, zs, mb);
        sv = member_ptr(sv, zs, mb);
        gd = member_ptr(gd, zs, mb);
    }
    __shared__ int red_k, red_nd, red_nr;
    const int q = blockIdx.x, t = threadIdx.x;
    const MergeGeo g = merge_geo(level, q, n, nl);
    const int a = g.a, n1 = g.m - g.a, n2 = g.b - g.m, nm = g.b - g.a;
    const bool flagged = status[2] == ST_ENONFINITE;
    const double beta = flagged ? 0.0 : e[g.m - 1];
    double rho = 2.0 * fabs(beta);
    const double sgn = beta < 0.0 ? -1.0 : 1.0;
    const double rs2 = 0.70710678118654752440;
    double *z = dv + (int64_t)DZ * n + a, *Dm = dv + (int64_t)DDM * n + a, *dd = dv + (int64_t)DDD * n + a;
    double *dh = dv + (int64_t)DDH * n + a, *zh = dv + (int64_t)DZH * n + a;
    double *rcs = dv + (int64_t)DRC * n + a, *rsn = dv + (int64_t)DRS * n + a;
    int *perm = iv + (int64_t)IPERM * n + a, *keep = iv + (int64_t)IKEEP * n + a;
    int *defl = iv + (int64_t)IDEFL * n + a, *rp = iv + (int64_t)IRP * n + a, *rn = iv + (int64_t)IRN * n + a;
    int *rowk = iv + (int64_t)IROWK * n + a;
    // Every value must compare for the ranks and the deflation below to index
    // correctly; a merge that meets a NaN or an infinity (flagged input, or
    // overflow) is carried out on zeros instead and the block is flagged, so
    // the rest of the solver stays in bounds (the output becomes NaN).
    bool finite = isfinite(rho);
    for (int i = t; i < nm; i += blockDim.x) {
        const double zi = (i < n1) ? Qcur[(g.m - 1) + (int64_t)(a + i) * ldq] * rs2
                                   : sgn * Qcur[g.m + (int64_t)(g.m + i - n1) * ldq] * rs2;
        const double di = Dcur[a + i];
        finite = finite && isfinite(zi) && isfinite(di);
        z[i] = zi;
        Dm[i] = di;
        dd[i] = di;
    }
    const bool sane = __syncthreads_and(finite ? 1 : 0) != 0;
    if (!sane) {
        rho = 0.0;
        for (int i = t; i < nm; i += blockDim.x) { z[i] = 0.0; Dm[i] = 0.0; dd[i] = 0.0; }
        if (t == 0 && status[2] == ST_OK) status[2] = ST_ENONFINITE;
        __syncthreads();
    }
    double zmax = 0.0, dmax = 0.0;
    for (int i = t; i < nm; i += blockDim.x) {
        zmax = fmax(zmax, fabs(z[i]));
        dmax = fmax(dmax, fabs(dd[i]));
    }
    // block max via the sum helper on a two-pass scheme
    {
        __shared__ double mx[2][4];
        double v1 = zmax, v2 = dmax;
        for (int o = 32; o > 0; o >>= 1) {
            v1 = fmax(v1, __shfl_xor(v1, o, 64));
            v2 = fmax(v2, __shfl_xor(v2, o, 64));
        }
        if ((t & 63) == 0) { mx[0][t >> 6] = v1; mx[1][t >> 6] = v2; }
        __syncthreads();
        zmax = fmax(fmax(mx[0][0], mx[0][1]), fmax(mx[0][2], mx[0][3]));
        dmax = fmax(fmax(mx[1][0], mx[1][1]), fmax(mx[1][2], mx[1][3]));
    }
    // The sequential merge/deflation scan runs on LDS copies when they fit.
    extern __shared__ __align__(16) unsigned char prep_lds[];
    const bool in_lds = use_lds != 0;  // the launch sized the LDS for the largest merge
    double *zl = in_lds ? reinterpret_cast<double *>(prep_lds) : z;
    double *dl = in_lds ? zl + nm : dd;
    int *pl = in_lds ? reinterpret_cast<int *>(dl + nm) : perm;
    if (in_lds) {
        for (int i = t; i < nm; i += blockDim.x) { zl[i] = z[i]; dl[i] = dd[i]; }
    }
    __syncthreads();
    // Fast path, in parallel: merge the two ascending halves by ranks (ties:
    // the first half first), split the merged order into deflated (small z)
    // and kept entries, and test every consecutive kept pair for the
    // close-pair rotation with the scan's own expression.  When no pair
    // qualifies (and both halves are ascending) nothing rotates, and this is
    // exactly what the sequential scan below produces; otherwise the scan
    // runs from scratch.
    __shared__ int fast_ok;
    __shared__ int kcnt[256];
    const double tol = 8.0 * EPS * fmax(dmax, rho * zmax);
    if (t == 0) fast_ok = 1;
    __syncthreads();
    for (int i = t; i + 1 < nm; i += blockDim.x)
        if (i + 1 != n1 && dl[i + 1] < dl[i]) fast_ok = 0;
    for (int i = t; i < nm; i += blockDim.x) {
        const double v = dl[i];
        int pos;
        if (i < n1) {  // second-half values strictly below v
            int lo = n1, hi = nm;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (dl[mid] < v) lo = mid + 1; else hi = mid;
            }
            pos = i + (lo - n1);
        } else {  // first-half values at or below v
            int lo = 0, hi = n1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (dl[mid] <= v) lo = mid + 1; else hi = mid;
            }
            pos = (i - n1) + lo;
        }
        pl[pos] = i;  // in range whatever the data; overwritten by the scan if unsorted
    }
    __syncthreads();
    const int chunk = (nm + 255) / 256;
    const int cb0 = min(nm, t * chunk), cb1 = min(nm, cb0 + chunk);
    {
        int nk = 0;
        for (int idx = cb0; idx < cb1; ++idx) nk += (rho * fabs(zl[pl[idx]]) <= tol) ? 0 : 1;
        kcnt[t] = nk;
    }
    __syncthreads();
    if (t == 0) {
        int acc = 0;
        for (int u = 0; u < 256; ++u) {
            const int cu = kcnt[u];
            kcnt[u] = acc;
            acc += cu;
        }
        red_k = acc;
    }
    __syncthreads();
    {
        int kk = kcnt[t], nd0 = cb0 - kcnt[t];
        for (int idx = cb0; idx < cb1; ++idx) {
            const int p = pl[idx];
            if (rho * fabs(zl[p]) <= tol) defl[nd0++] = p;
            else keep[kk++] = p;
        }
    }
    __syncthreads();
    {
        const int kt = red_k;
        for (int i = 1 + t; i < kt; i += blockDim.x) {
            const int prev = keep[i - 1], p = keep[i];
            const double tz = hypot(zl[prev], zl[p]);
            const double c = zl[p] / tz, s = -zl[prev] / tz;
            const double tt = dl[p] - dl[prev];
            if (fabs(tt * c * s) <= tol) fast_ok = 0;
        }
    }
    __syncthreads();
    if (t == 0 && fast_ok) {
        red_nd = nm - red_k;
        red_nr = 0;
    }
    if (t == 0 && !fast_ok) {
        // merge the two ascending halves into one ascending order
        int i1 = 0, i2 = n1, o = 0;
        while (i1 < n1 && i2 < nm) pl[o++] = (dl[i2] < dl[i1]) ? i2++ : i1++;
        while (i1 < n1) pl[o++] = i1++;
        while (i2 < nm) pl[o++] = i2++;
        // deflation
        int k = 0, nd = 0, nr = 0, prev = -1;
        for (int idx = 0; idx < nm; ++idx) {
            const int p = pl[idx];
            if (rho * fabs(zl[p]) <= tol) { defl[nd++] = p; continue; }
            if (prev >= 0) {
                const double tz = hypot(zl[prev], zl[p]);
                const double c = zl[p] / tz, s = -zl[prev] / tz;
                const double tt = dl[p] - dl[prev];
                if (fabs(tt * c * s) <= tol) {
                    zl[p] = tz;
                    zl[prev] = 0.0;
                    const double dp = dl[prev] * c * c + dl[p] * s * s;
                    const double dn = dl[prev] * s * s + dl[p] * c * c;
                    dl[prev] = dp;
                    dl[p] = dn;
                    rp[nr] = prev; rn[nr] = p; rcs[nr] = c; rsn[nr] = s; ++nr;
                    defl[nd++] = prev;
                    --k;
                }
            }
            keep[k++] = p;
            prev = p;
        }
        red_k = k;
        red_nd = nd;
        red_nr = nr;
    }
    __syncthreads();
    const int k = red_k;
    // kept values / weights and the row -> kept-index map
    for (int i = t; i < nm; i += blockDim.x) rowk[i] = -1;
    __syncthreads();
    for (int i = t; i < k; i += blockDim.x) {
        const int p = keep[i];
        dh[i] = dl[p];
        zh[i] = zl[p];
        rowk[p] = i;
    }
    for (int i = t; i < nm; i += blockDim.x) dd[i] = dl[i];
    if (t == 0) {
        const int nd = red_nd, nr = red_nr;
        sv[q * SCOUNT + SK] = k;
        sv[q * SCOUNT + SND] = nd;
        sv[q * SCOUNT + SNR] = nr;
        dv[(int64_t)DRHO * n + q] = rho;
        // merge GEMMs: Qnext[a:m, a:b] = Q1 U[0:n1, :], Qnext[m:b, a:b] = Q2 U[n1:, :]
        GemmDesc top{}, bot{};
        top.M = n1; top.N = nm; top.K = n1;
        top.A = GemmOperand{Qcur + a + (int64_t)a * ldq, Qcur + a + (int64_t)a * ldq, ldq, ldq, n1, OP_N, nullptr};
        top.B = GemmOperand{U + (int64_t)a * n + a, U + (int64_t)a * n + a, n, n, n1, OP_C, nullptr};
        top.C = Qnext + a + (int64_t)a * ldq; top.ldc = ldq; top.alpha = 1.0; top.beta = 0.0;
        bot.M = n2; bot.N = nm; bot.K = n2;
        bot.A = GemmOperand{Qcur + g.m + (int64_t)g.m * ldq, Qcur + g.m + (int64_t)g.m * ldq, ldq, ldq, n2, OP_N, nullptr};
        bot.B = GemmOperand{U + (int64_t)g.m * n + a, U + (int64_t)g.m * n + a, n, n, n2, OP_C, nullptr};
        bot.C = Qnext + g.m + (int64_t)a * ldq; bot.ldc = ldq; bot.alpha = 1.0; bot.beta = 0.0;
        gd[2 * q] = top;
        gd[2 * q + 1] = bot;
    }
}

// Product of one double over a wave whose lanes are all active, the same in
// every lane: the exchange pattern of wave_sum_dpp with products.
__device__ __forceinline__ double wave_prod_dpp(double v) {
    v *= dpp_double<0xB1>(v);
    v *= dpp_double<0x4E>(v);
    v *= dpp_double<0x141>(v);
    v *= dpp_double<0x140>(v);
    return ((readlane_double(v, 0) * readlane_double(v, 16)) * readlane_double(v, 32)) * readlane_double(v, 48);
}

// Root j of 1 + rho sum_i zh_i^2 / (dh_i - lambda) = 0 (dh ascending, gaps
// > 0), solved by one wave (every lane active): the lanes split every sum
// over i and the wave-wide DPP sums give all lanes the same totals, so all
// lanes take the same steps.  Returns the origin pole o and tau with lambda = dh[o] + tau.
__device__ bool secular_root_wave(const double *dh, const double *zh, int k, double rho, int j, int *o_out,
                                  double *tau_out) {
    const int lane = threadIdx.x & 63;
    int o;
    double lo, hi;
    if (j < k - 1) {
        const double gap = dh[j + 1] - dh[j];
        double f = 0.0;
        for (int i = lane; i < k; i += 64) f += rho * zh[i] * zh[i] / ((dh[i] - dh[j]) - 0.5 * gap);
        f = 1.0 + wave_sum_dpp(f);
        if (f > 0.0) { o = j; lo = 0.0; hi = 0.5 * gap; }
        else { o = j + 1; lo = -0.5 * gap; hi = 0.0; }
    } else {
        double zz = 0.0;
        for (int i = lane; i < k; i += 64) zz += zh[i] * zh[i];
        zz = wave_sum_dpp(zz);
        o = j; lo = 0.0; hi = rho * zz;
    }
    const double dO = dh[o];
    double tau = 0.5 * (lo + hi);
    bool converged = false;
    for (int it = 0; it < 100; ++it) {
        double psi = 0.0, phi = 0.0, dpsi = 0.0, dphi = 0.0, sabs = 0.0;
        for (int i = lane; i < k; i += 64) {
            const double diff = (dh[i] - dO) - tau;
            const double w = rho * zh[i] * zh[i];
            const double term = w / diff;
            sabs += fabs(term);
            if (i <= j) { psi += term; dpsi += term / diff; }
            else { phi += term; dphi += term / diff; }
        }
        psi = wave_sum_dpp(psi); phi = wave_sum_dpp(phi);
        dpsi = wave_sum_dpp(dpsi); dphi = wave_sum_dpp(dphi); sabs = wave_sum_dpp(sabs);
        const double f = 1.0 + psi + phi;
        if (f < 0.0) lo = tau; else hi = tau;
        if (f == 0.0 || fabs(f) <= 8.0 * EPS * (1.0 + sabs)) { converged = true; break; }
        if (hi - lo <= 2.0 * EPS * fmax(fabs(lo), fabs(hi))) { converged = true; break; }
        const double a_ = (dh[j] - dO) - tau;
        double tn;
        bool ok = false;
        if (j < k - 1) {
            const double b_ = (dh[j + 1] - dO) - tau;
            const double s = dpsi * a_ * a_, S = dphi * b_ * b_;
            const double c = f - s / a_ - S / b_;
            const double B = c * (a_ + b_) + s + S;
            const double disc = B * B - 4.0 * c * f * a_ * b_;
            double eta = 0.0;
            if (disc >= 0.0) {
                const double sq = sqrt(disc);
                if (c == 0.0) { if (B != 0.0) { eta = f * a_ * b_ / B; ok = true; } }
                else if (B > 0.0) { eta = 2.0 * f * a_ * b_ / (B + sq); ok = true; }
                else { eta = (B - sq) / (2.0 * c); ok = true; }
            }
            tn = tau + eta;
        } else {
            const double s = dpsi * a_ * a_;
            const double c = 1.0 + phi + psi - s / a_;
            tn = tau + a_ + s / c;
            ok = c > 0.0;
        }
        if (!ok || !(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (fabs(tn - tau) <= 2.0 * EPS * fabs(tn)) { tau = tn; converged = true; break; }
        tau = tn;
    }
    *o_out = o;
    *tau_out = tau;
    return converged;
}

// One wave per root: 4 roots per 256-thread workgroup.
__global__ void __launch_bounds__(256) dc_secular_kernel(int level, int n, int nl, double *dv, int *iv,
                                                         const int *sv, int *status, int64_t zs) {
    {
        const int mb = blockIdx.z;
        status = member_ptr(status, zs, mb);
        dv = member_ptr(dv, zs, mb);
        iv = member_ptr(iv, zs, mb);
        sv = member_ptr(sv, zs, mb);
    }
    const int q = blockIdx.y;
    const MergeGeo g = merge_geo(level, q, n, nl);
    const int a = g.a;
    const int k = sv[q * SCOUNT + SK];
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= k) return;
    const double rho = dv[(int64_t)DRHO * n + q];
    const double *dh = dv + (int64_t)DDH * n + a, *zh = dv + (int64_t)DZH * n + a;
    int o;
    double tau;
    const bool converged = secular_root_wave(dh, zh, k, rho, j, &o, &tau);
    if ((threadIdx.x & 63) == 0) {
        if (!converged && status[2] == ST_OK) status[2] = ST_ENOCONV;
        iv[(int64_t)IORG * n + a + j] = o;
        dv[(int64_t)DTAU * n + a + j] = tau;
        dv[(int64_t)DLAM * n + a + j] = dh[o] + tau;
    }
}

// zhat_i^2 = prod_j (lambda_j - d_i) / (rho prod_{l != i} (d_l - d_i)), paired
// so that every factor is a ratio in (0, 1] (interlacing).
__global__ void __launch_bounds__(256) dc_lowner_kernel(int level, int n, int nl, double *dv, const int *iv,
                                                        const int *sv, int64_t zs) {
    {
        const int mb = blockIdx.z;
        dv = member_ptr(dv, zs, mb);
        iv = member_ptr(iv, zs, mb);
        sv = member_ptr(sv, zs, mb);
    }
    const int q = blockIdx.y;
    const MergeGeo g = merge_geo(level, q, n, nl);
    const int a = g.a;
    const int k = sv[q * SCOUNT + SK];
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= k) return;
    const double rho = dv[(int64_t)DRHO * n + q];
    const double *dh = dv + (int64_t)DDH * n + a, *zh = dv + (int64_t)DZH * n + a;
    const double *tau = dv + (int64_t)DTAU * n + a;
    const int *org = iv + (int64_t)IORG * n + a;
    const double di = dh[i];
    // each factor is a ratio in (0, 1]; lanes multiply disjoint subsets
    double prod = 1.0;
    for (int jj = lane; jj < k - 1; jj += 64) {
        const double num = (dh[org[jj]] - di) + tau[jj];
        const double den = (jj < i) ? (dh[jj] - di) : (dh[jj + 1] - di);
        prod *= num / den;
    }
    prod = wave_prod_dpp(prod) * (((dh[org[k - 1]] - di) + tau[k - 1]) / rho);
    if (lane == 0) dv[(int64_t)DZHAT * n + a + i] = copysign(sqrt(fmax(prod, 0.0)), zh[i]);
}

// Norm of the secular eigenvector of root j: one wave per root.
__global__ void __launch_bounds__(256) dc_norm_kernel(int level, int n, int nl, double *dv, const int *iv,
                                                      const int *sv, int64_t zs) {
    {
        const int mb = blockIdx.z;
        dv = member_ptr(dv, zs, mb);
        iv = member_ptr(iv, zs, mb);
        sv = member_ptr(sv, zs, mb);
    }
    const int q = blockIdx.y;
    const MergeGeo g = merge_geo(level, q, n, nl);
    const int a = g.a;
    const int k = sv[q * SCOUNT + SK];
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= k) return;
    const double *dh = dv + (int64_t)DDH * n + a, *zhat = dv + (int64_t)DZHAT * n + a;
    const int o = iv[(int64_t)IORG * n + a + j];
    const double tj = dv[(int64_t)DTAU * n + a + j], dO = dh[o];
    double s2 = 0.0;
    for (int i = lane; i < k; i += 64) {
        const double u = zhat[i] / ((dh[i] - dO) - tj);
        s2 += u * u;
    }
    s2 = wave_sum_dpp(s2);
    if (lane == 0) dv[(int64_t)DNRM * n + a + j] = 1.0 / sqrt(s2);
}

// Final ascending order of the merged eigenvalues (secular roots + deflated
// values); ties broken by element id.  Writes the eigenvalues and, per final
// column, its source (j >= 0: root j; -(1+p): deflated local index p).
__global__ void __launch_bounds__(256) dc_order_kernel(int level, int n, int nl, const double *dv, int *iv,
                                                       const int *sv, double *Dnext, int64_t zs) {
    {
        const int mb = blockIdx.z;
        dv = member_ptr(dv, zs, mb);
        iv = member_ptr(iv, zs, mb);
        sv = member_ptr(sv, zs, mb);
        Dnext = member_ptr(Dnext, zs, mb);
    }
    const int q = blockIdx.y;
    const MergeGeo g = merge_geo(level, q, n, nl);
    const int a = g.a, nm = g.b - g.a;
    const int k = sv[q * SCOUNT + SK], nd = sv[q * SCOUNT + SND];
    const int el = blockIdx.x * blockDim.x + threadIdx.x;
    if (el >= nm) return;
    const double *lam = dv + (int64_t)DLAM * n + a, *dd = dv + (int64_t)DDD * n + a;
    const int *defl = iv + (int64_t)IDEFL * n + a;
    const double v = el < k ? lam[el] : dd[defl[el - k]];
    // roots (value, id) are lexicographically ascending: binary search
    int lo = 0, hi = k;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const bool less = lam[mid] < v || (lam[mid] == v && mid < el);
        if (less) lo = mid + 1; else hi = mid;
    }
    int rank = lo;
    for (int p = 0; p < nd; ++p) {
        const double u = dd[defl[p]];
        rank += (u < v) || (u == v && k + p < el);
    }
    iv[(int64_t)ICOL * n + a + rank] = el < k ? el : -(1 + defl[el - k]);
    Dnext[a + rank] = v;
}

// U[r][col] of the merge matrix (row-major, ld n, block at (a, a)), one
// element per thread: column col holds the normalised secular vector of a
// root (rows of the kept poles) or the unit vector of a deflated pole.
__global__ void __launch_bounds__(256) dc_vectors_kernel(int level, int n, int nl, const double *dv,
                                                         const int *iv, const int *sv, double *U, int64_t zs) {
    const int nmerge = nl >> level;
    const int mb = blockIdx.z / nmerge, q = blockIdx.z - mb * nmerge;
    dv = member_ptr(dv, zs, mb);
    iv = member_ptr(iv, zs, mb);
    sv = member_ptr(sv, zs, mb);
    U = member_ptr(U, zs, mb);
    const MergeGeo g = merge_geo(level, q, n, nl);
    const int a = g.a, nm = g.b - g.a;
    const int k = sv[q * SCOUNT + SK];
    const int col = blockIdx.x * 64 + (threadIdx.x & 63);
    const int r = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (col >= nm || r >= nm) return;
    const double *dh = dv + (int64_t)DDH * n + a, *zhat = dv + (int64_t)DZHAT * n + a;
    const double *tau = dv + (int64_t)DTAU * n + a, *nrm = dv + (int64_t)DNRM * n + a;
    const int *org = iv + (int64_t)IORG * n + a, *rowk = iv + (int64_t)IROWK * n + a;
    const int src = iv[(int64_t)ICOL * n + a + col];
    double u = 0.0;
    if (src >= 0 && src < k) {
        const int i = rowk[r];
        if (i >= 0 && i < k) {
            const int o = org[src];
            u = zhat[i] / ((dh[i] - dh[o]) - tau[src]) * nrm[src];
        }
    } else if (src < 0 && -1 - src == r) {
        u = 1.0;
    }
    U[(int64_t)(a + r) * n + a + col] = u;
}

// Undo the deflating rotations (last first) on the rows of U, one column per
// thread.
__global__ void __launch_bounds__(256) dc_rotate_kernel(int level, int n, int nl, const double *dv, const int *iv,
                                                        const int *sv, double *U, int64_t zs) {
    {
        const int mb = blockIdx.z;
        dv = member_ptr(dv, zs, mb);
        iv = member_ptr(iv, zs, mb);
        sv = member_ptr(sv, zs, mb);
        U = member_ptr(U, zs, mb);
    }
    const int q = blockIdx.y;
    const MergeGeo g = merge_geo(level, q, n, nl);
    const int a = g.a, nm = g.b - g.a;
    const int nr = sv[q * SCOUNT + SNR];
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= nm || nr == 0) return;
    const double *rcs = dv + (int64_t)DRC * n + a, *rsn = dv + (int64_t)DRS * n + a;
    const int *rp = iv + (int64_t)IRP * n + a, *rn = iv + (int64_t)IRN * n + a;
    double *Uc = U + (int64_t)a * n + a + col;  // U[r][col] = Uc[r * n]
    for (int r = nr - 1; r >= 0; --r) {
        const int pp = rp[r], pn = rn[r];
        const double c = rcs[r], s = rsn[r];
        const double up = Uc[(int64_t)pp * n], un = Uc[(int64_t)pn * n];
        Uc[(int64_t)pp * n] = c * up - s * un;
        Uc[(int64_t)pn * n] = s * up + c * un;
    }
}

int dc_num_leaves(int n) {
    int nl = 1;
    while ((n + nl - 1) / nl > DC_LEAF) nl <<= 1;
    return nl;
}

}  // namespace

hipError_t dc_prepare() {
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)dc_prep_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           PREP_LDS_MAX * 20);
        if (e != hipSuccess) return e;
        attr = true;
    }
    return hipSuccess;
}

hipError_t large_dc(LargeWs &w, hipStream_t st) {
    {
        hipError_t e = dc_prepare();
        if (e != hipSuccess) return e;
    }
    const int n = w.n;
    const int nl = dc_num_leaves(n);
    int64_t ldq = n;
    double *Qc = w.Q0, *Qn = w.Q1, *Dc = w.D0, *Dn = w.D1;
    const int B = w.nmem;
    const int64_t zs = w.zs;
    hipLaunchKernelGGL(dc_leaf_kernel, dim3(nl, 1, B), dim3(64), 0, st, w.d, w.e, n, nl, Dc, Qc, ldq, w.ksel, zs);
    for (int level = 1; (1 << level) <= nl; ++level) {
        const int nmerge = nl >> level;
        int maxnm = 0, maxhalf = 0;
        for (int q = 0; q < nmerge; ++q) {
            const int a = leaf_bound(q << level, n, nl), m = leaf_bound((q << level) + (1 << (level - 1)), n, nl),
                      b = leaf_bound((q + 1) << level, n, nl);
            maxnm = std::max(maxnm, b - a);
            maxhalf = std::max(maxhalf, std::max(m - a, b - m));
        }
        const int use_lds = maxnm <= PREP_LDS_MAX ? 1 : 0;
        const size_t prep_lds = use_lds ? (size_t)maxnm * 20 : 0;
        hipLaunchKernelGGL(dc_prep_kernel, dim3(nmerge, 1, B), dim3(256), prep_lds, st, level, n, nl, w.e, Dc, Qc,
                           Qn, ldq, w.U, w.dcd, w.dci, w.dcs, w.gdesc, use_lds, w.ksel, zs);
        dim3 wgrid((maxnm + 3) / 4, nmerge, B);
        dim3 tgrid((maxnm + 255) / 256, nmerge, B);
        hipLaunchKernelGGL(dc_secular_kernel, wgrid, dim3(256), 0, st, level, n, nl, w.dcd, w.dci, w.dcs, w.ksel,
                           zs);
        hipLaunchKernelGGL(dc_lowner_kernel, wgrid, dim3(256), 0, st, level, n, nl, w.dcd, w.dci, w.dcs, zs);
        hipLaunchKernelGGL(dc_norm_kernel, wgrid, dim3(256), 0, st, level, n, nl, w.dcd, w.dci, w.dcs, zs);
        hipLaunchKernelGGL(dc_order_kernel, tgrid, dim3(256), 0, st, level, n, nl, w.dcd, w.dci, w.dcs, Dn, zs);
        dim3 vgrid((maxnm + 63) / 64, (maxnm + 3) / 4, nmerge * B);
        hipLaunchKernelGGL(dc_vectors_kernel, vgrid, dim3(256), 0, st, level, n, nl, w.dcd, w.dci, w.dcs, w.U, zs);
        hipLaunchKernelGGL(dc_rotate_kernel, tgrid, dim3(256), 0, st, level, n, nl, w.dcd, w.dci, w.dcs, w.U, zs);
        hipError_t e = gemm_launch_batched(w.gdesc, 2 * nmerge, maxhalf, maxnm, false, st, B, zs);
        if (e != hipSuccess) return e;
        std::swap(Qc, Qn);
        std::swap(Dc, Dn);
    }
    w.lam = Dc;
    w.Zfinal = Qc;
    return hipGetLastError();
}

}  // namespace psd
