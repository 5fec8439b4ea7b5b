// Whole-block projection of small Hermitian blocks (order n <= 64) by one
// workgroup entirely in LDS.  Serves single blocks of order <= 64 (e.g. the
// d=2 process matrix, n=16) and the instrument Choi blocks (d^2 x d^2) of a
// batched cone.
//
// Steps, all in LDS (M = conj X, column-major, see common.h):
//   1. unpack the svec block (App. D.1 vec_R) into the full Hermitian M;
//   2. two-sided Jacobi M <- U^H M U, V <- V U, until M is diagonal: each
//      step applies n/2 disjoint plane rotations at once (round-robin
//      pairing, every pair once per sweep), each a phase on index q that
//      makes M(p,q) real followed by the real rotation that zeroes it;
//      rotations below the relative threshold eps sqrt(|M(p,p)| |M(q,q)|)
//      are skipped, and the iteration stops after a sweep without one;
//   3. Pi = V+ diag(lambda+) V+^H, or X + V- diag(|lambda-|) V-^H when fewer
//      eigenvalues are non-positive (App. D.2: eigendecompose, zero the
//      negative eigenvalues), written straight back as svec.
// Every step is n/2 independent rotations over the 256 threads: a few
// dozen barrier-separated steps per sweep, where a tridiagonal QL computes
// its rotations one after another.  Blocks of order <= 32 take a form with
// one barrier per step (small32_project_kernel below).
#include "common.h"
#include "kernels.h"

namespace psd {

constexpr int SB_MAX = 64;     // largest order served
constexpr int SB_LD = 65;      // LDS leading dimension (odd: row and column walks spread over the banks)
constexpr int SB_NT = 256;     // threads per workgroup
constexpr int SB_SWEEPS = 40;  // sweeps before reporting non-convergence

struct SmallLds {
    cd A[SB_LD * SB_MAX];  // M, rotated towards diagonal form
    cd V[SB_LD * SB_MAX];  // accumulated rotations: eigenvectors in the columns
    // rotation of pair k of the current step: columns p, q, cosine, sine,
    // phase e^{i phi} of M(p, q), and the new diagonal entries
    int rp[SB_MAX / 2 + 1], rq[SB_MAX / 2 + 1];
    double rc[SB_MAX / 2 + 1], rs[SB_MAX / 2 + 1], rdp[SB_MAX / 2 + 1], rdq[SB_MAX / 2 + 1];
    cd rph[SB_MAX / 2 + 1];
    int ract[SB_MAX / 2 + 1];
    double lam[SB_MAX], scal[SB_MAX];
    int perm[SB_MAX];
    int sel[SB_MAX];
    int rotated, status, ksel, sgn;
};

// Pair k of round r of the round-robin over m (even) indices: index m - 1 is
// fixed, the others turn; every pair occurs once in rounds 0 .. m-2.
__device__ __forceinline__ void rr_pair(int m, int r, int k, int &p, int &q) {
    int a, b;
    if (k == 0) {
        a = r;
        b = m - 1;
    } else {
        a = (r + k) % (m - 1);
        b = (r - k + (m - 1)) % (m - 1);
    }
    p = min(a, b);
    q = max(a, b);
}

// Two-sided Jacobi of the Hermitian S.A (order n), V = I on entry.
__device__ void small_jacobi(SmallLds &S, int n) {
    const int t = threadIdx.x;
    const double eps = 2.220446049250313e-16;
    const int m = n + (n & 1);  // an odd order gets a dummy index n that never rotates
    const int npairs = m / 2;
    int sweep = 0;
    for (; sweep < SB_SWEEPS; ++sweep) {
        if (t == 0) S.rotated = 0;
        __syncthreads();
        for (int r = 0; r + 1 < m; ++r) {
            // 1. rotation parameters, one thread per pair, from the current M
            if (t < npairs) {
                int p, q;
                rr_pair(m, r, t, p, q);
                S.rp[t] = p;
                S.rq[t] = q;
                int act = 0;
                if (q < n) {
                    const cd apq = S.A[p + q * SB_LD];
                    const double app = S.A[p + p * SB_LD].x, aqq = S.A[q + q * SB_LD].x;
                    const double rr = sqrt(cabs2(apq));
                    if (rr > 0.0 && rr > eps * sqrt(fabs(app) * fabs(aqq))) {
                        act = 1;
                        const cd ph = cmk(apq.x / rr, apq.y / rr);  // e^{i phi}
                        const double tau = (aqq - app) / (2.0 * rr);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        const double c = 1.0 / sqrt(1.0 + tt * tt);
                        S.rc[t] = c;
                        S.rs[t] = tt * c;
                        S.rph[t] = ph;
                        S.rdp[t] = app - tt * rr;
                        S.rdq[t] = aqq + tt * rr;
                        S.rotated = 1;  // benign race: all writers store 1
                    }
                }
                S.ract[t] = act;
            }
            __syncthreads();
            // 2. rows p, q of every active pair: (U^H M) with U = D J,
            //    D = diag(1, conj(ph)) on q, J = [[c, s], [-s, c]]
            for (int idx = t; idx < npairs * n; idx += SB_NT) {
                const int k = idx / n, col = idx % n;
                if (!S.ract[k]) continue;
                const int p = S.rp[k], q = S.rq[k];
                const double c = S.rc[k], sn = S.rs[k];
                const cd ph = S.rph[k];
                const cd ap = S.A[p + col * SB_LD], aq = cmul(ph, S.A[q + col * SB_LD]);
                S.A[p + col * SB_LD] = cmk(c * ap.x - sn * aq.x, c * ap.y - sn * aq.y);
                S.A[q + col * SB_LD] = cmk(sn * ap.x + c * aq.x, sn * ap.y + c * aq.y);
            }
            __syncthreads();
            // 3. columns p, q of M and V: (M U), (V U); the 2x2 block of each
            //    pair set to its exact diagonal form
            for (int idx = t; idx < npairs * n; idx += SB_NT) {
                const int k = idx / n, row = idx % n;
                if (!S.ract[k]) continue;
                const int p = S.rp[k], q = S.rq[k];
                const double c = S.rc[k], sn = S.rs[k];
                const cd phc = cconj(S.rph[k]);
                {
                    const cd ap = S.A[row + p * SB_LD], aq = cmul(phc, S.A[row + q * SB_LD]);
                    cd np = cmk(c * ap.x - sn * aq.x, c * ap.y - sn * aq.y);
                    cd nq = cmk(sn * ap.x + c * aq.x, sn * ap.y + c * aq.y);
                    if (row == p) { np = cmk(S.rdp[k], 0.0); nq = cmk(0.0, 0.0); }
                    if (row == q) { np = cmk(0.0, 0.0); nq = cmk(S.rdq[k], 0.0); }
                    S.A[row + p * SB_LD] = np;
                    S.A[row + q * SB_LD] = nq;
                }
                {
                    const cd vp = S.V[row + p * SB_LD], vq = cmul(phc, S.V[row + q * SB_LD]);
                    S.V[row + p * SB_LD] = cmk(c * vp.x - sn * vq.x, c * vp.y - sn * vq.y);
                    S.V[row + q * SB_LD] = cmk(sn * vp.x + c * vq.x, sn * vp.y + c * vq.y);
                }
            }
            __syncthreads();
        }
        const int any = S.rotated;
        __syncthreads();
        if (!any) break;
    }
    if (t == 0 && sweep == SB_SWEEPS && S.status == ST_OK) S.status = ST_ENOCONV;
    __syncthreads();
}

// Unpack the svec block into the full Hermitian S.A (leading dimension LD)
// and set S.V = I.  Non-finite input: NaN in every output entry, the info
// record says so, and false is returned (every thread alike).
template <int LD, class Lds>
__device__ bool small_unpack(Lds &S, const SmallJob &job, const double *x, double *y, psd_dev_info *infos) {
    const int n = job.n, t = threadIdx.x;
    const double rs2 = 0.70710678118654752440;
    if (t == 0) S.status = ST_OK;
    __syncthreads();
    // lower triangle of M from the svec columns, mirrored
    int bad = 0;
    for (int idx = t; idx < n * n; idx += (int)blockDim.x) {
        const int i = idx % n, j = idx / n;
        if (i < j) continue;
        cd v;
        if (i == j) {
            v = cmk(x[svec_col_start(n, j)], 0.0);
        } else {
            const long o = svec_off(n, i, j);
            v = cmk(x[o] * rs2, x[o + 1] * rs2);
        }
        bad |= !(isfinite(v.x) && isfinite(v.y));
        S.A[i + j * LD] = v;
        S.A[j + i * LD] = cconj(v);
    }
    for (int idx = t; idx < n * n; idx += (int)blockDim.x) {
        const int i = idx % n, j = idx / n;
        S.V[i + j * LD] = cmk((i == j) ? 1.0 : 0.0, 0.0);
    }
    if (bad) S.status = ST_ENONFINITE;  // benign race: all writers store the same value
    __syncthreads();
    if (S.status == ST_OK) return true;
    // the projection is undefined: report it and return NaN in every entry
    for (int idx = t; idx < n * n; idx += (int)blockDim.x) {
        const int i = idx % n, j = idx / n;
        if (i < j) continue;
        if (i == j) y[svec_col_start(n, j)] = __builtin_nan("");
        else { const long o = svec_off(n, i, j); y[o] = __builtin_nan(""); y[o + 1] = __builtin_nan(""); }
    }
    if (t == 0 && infos) {
        psd_dev_info &I = infos[job.info_index];
        I.status = ST_ENONFINITE; I.n_pos = 0; I.n_neg = 0; I.iters = 0; I.fallback = 0; I.est_rel_err = 0.0;
        I.scale = 0.0;
    }
    return false;
}

// After the rotations: eigenvalues = diag S.A, eigenvectors = columns of
// S.V.  Sort, pick the smaller sign side, write the info record, the
// optional saved eigenpairs, and the projection as svec.
template <int LD, class Lds>
__device__ void small_finish(Lds &S, const SmallJob &job, const double *x, double *y, psd_dev_info *infos,
                             double *saved_all) {
    const int n = job.n, t = threadIdx.x;
    // ascending order of the eigenvalues (the diagonal of the rotated M)
    if (t < n) {
        const double v = S.A[t + t * LD].x;
        int rank = 0;
        for (int q = 0; q < n; ++q) {
            const double u = S.A[q + q * LD].x;
            rank += (u < v) || (u == v && q < t);
        }
        S.lam[rank] = v;
        S.perm[rank] = t;  // column of V
    }
    __syncthreads();
    if (t == 0) {
        int npos = 0;
        for (int q = 0; q < n; ++q) npos += S.lam[q] > 0.0;
        const int nneg = n - npos;
        // project on the smaller side
        if (npos <= nneg) { S.ksel = npos; S.sgn = 1; for (int q = 0; q < npos; ++q) S.sel[q] = S.perm[n - npos + q]; }
        else { S.ksel = nneg; S.sgn = -1; for (int q = 0; q < nneg; ++q) S.sel[q] = S.perm[q]; }
        for (int q = 0; q < S.ksel; ++q) {
            const int rk = S.sgn > 0 ? n - S.ksel + q : q;
            S.scal[q] = S.lam[rk];
        }
        if (infos) {
            psd_dev_info &I = infos[job.info_index];
            I.status = S.status; I.n_pos = npos; I.n_neg = nneg;
            I.iters = 0; I.fallback = 0; I.est_rel_err = 0.0; I.scale = 0.0;
        }
    }
    __syncthreads();

    // optional: full eigenvectors (ascending eigenvalues) for a later derivative
    if (saved_all) {
        double *sv = saved_all + job.saved_offset;
        if (t < n) sv[t] = S.lam[t];
        cd *V = reinterpret_cast<cd *>(sv + n);
        for (int idx = t; idx < n * n; idx += (int)blockDim.x) {
            const int r = idx % n, c = idx / n;
            V[r + (long)c * n] = S.V[r + S.perm[c] * LD];
        }
    }

    const int k = S.ksel;
    // reconstruct the lower triangle and pack.  Each thread reads x and
    // writes y at the same svec positions, so y may alias x.
    //   sgn>0: Pi = sum_{lambda>0} lambda v v^H;
    //   sgn<0: Pi = X - sum_{lambda<=0} lambda v v^H.
    const int sgn = S.sgn;
    const double sd = sgn > 0 ? 1.0 : -1.0;
    const double so = sd * 1.41421356237309504880;
    for (int idx = t; idx < n * n; idx += (int)blockDim.x) {
        const int i = idx % n, j = idx / n;
        if (i < j) continue;
        cd acc = cmk(0.0, 0.0);
        for (int c = 0; c < k; ++c) {
            const int col = S.sel[c];
            acc = cfma(cscale(S.V[i + col * LD], S.scal[c]), cconj(S.V[j + col * LD]), acc);
        }
        if (i == j) {
            const long o = svec_col_start(n, j);
            const double base = sgn > 0 ? 0.0 : x[o];
            y[o] = base + sd * acc.x;
        } else {
            const long o = svec_off(n, i, j);
            const double b0 = sgn > 0 ? 0.0 : x[o], b1 = sgn > 0 ? 0.0 : x[o + 1];
            y[o] = b0 + so * acc.x;
            y[o + 1] = b1 + so * acc.y;
        }
    }
}

__global__ void __launch_bounds__(SB_NT)
small_project_kernel(const SmallJob *jobs, SmallJob single, const double *__restrict__ xall,
                     double *yall, psd_dev_info *infos, double *saved_all) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    SmallLds &S = *reinterpret_cast<SmallLds *>(lds_raw);
    const SmallJob job = jobs ? jobs[blockIdx.x] : single;
    const double *x = xall + job.offset;
    double *y = yall + job.offset;
    if (!small_unpack<SB_LD>(S, job, x, y, infos)) return;
    small_jacobi(S, job.n);
    small_finish<SB_LD>(S, job, x, y, infos, saved_all);
}

// ---- Blocks of order <= 32: one barrier per Jacobi step ---------------------
//
// The same two-sided Jacobi (round-robin pairs, a phase then the real
// rotation, the 2x2 block of each rotated pair set to its exact diagonal
// form), arranged so that a step costs one barrier.  With M <- U^H M U and
// U block-diagonal over the step's n/2 pairs, entry (i, j) of M only
// depends on the 2x2 block of M at (pair of i, pair of j) and on those two
// rotations, and entry (i, j) of V <- V U on V(i, pair of j): all n/2 x n/2
// blocks are updated at once, four threads per block (one per entry) up to
// order 16, one thread per block above.  The
// next step's rotation of a pair (p', q') needs the new M(p', p'),
// M(q', q') -- the exact diagonal entries of this step's pairs, already
// known -- and the new M(p', q'), whose thread forms the rotation right
// after computing it.  Rotation records are double-buffered by step.
//
// Stopping: the projection is 1-Lipschitz in the Frobenius norm and U is
// unitary, so projecting the diagonal part of the rotated M (the
// eigenvalue estimates, with V) errs by at most the Frobenius norm of its
// off-diagonal part.  A sweep ends the iteration when that norm is at most
// SJ_TOL ||X||_F, or when no rotation passed the skip threshold -- the
// rule of the larger kernel, which needs one more sweep.
constexpr int SJ_MAX = 32;   // largest order served
constexpr int SJ_LD = 33;    // LDS leading dimension
constexpr int SJ_PAIRS = SJ_MAX / 2;
constexpr int SJ_NT = 256;   // largest workgroup (see sj_threads)
constexpr double SJ_TOL = 1e-14;

struct SjRot {
    double c, s, phx, phy, dp, dq;  // rotation, phase e^{i phi} of M(p, q), new diagonal entries
    int p, q, act, pad;
};

struct SmallLds32 {
    cd A[SJ_LD * SJ_MAX];
    cd V[SJ_LD * SJ_MAX];
    SjRot rot[2][SJ_PAIRS];
    unsigned char partner[SJ_MAX - 1][SJ_MAX];  // step r of a sweep: partner of index i
    unsigned char pairof[SJ_MAX - 1][SJ_MAX];   // step r: number of the pair holding index i
    double red[2][SJ_NT / 64];
    double lam[SJ_MAX], scal[SJ_MAX];
    int perm[SJ_MAX], sel[SJ_MAX];
    int rotated[3];
    int status, ksel, sgn;
};

// threads of the workgroup for order n: 4 per 2x2 block up to order 16,
// then one per block, in whole waves
__host__ __device__ inline int sj_threads(int n) {
    const int np = (n + (n & 1)) / 2;
    const int need = np <= 8 ? 4 * np * np : np * np;
    return need <= 64 ? 64 : (need + 63) / 64 * 64;
}

// 1/sqrt(x) and 1/x for x > 0 in FP64: the hardware estimates refined by
// two Newton steps (each at least doubles the correct bits), a short
// dependent chain where the rotation's divisions and square roots sit on
// every step's critical path.
__device__ __forceinline__ double sj_rsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return y;
}
__device__ __forceinline__ double sj_rcp(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    y = fma(y, fma(-x, y, 1.0), y);
    return y;
}

// Rotation of pair (p, q) from M(p, q), M(p, p), M(q, q): the formulas and
// skip rule of the larger kernel (|M(p, q)| <= eps sqrt(|M(p,p) M(q,q)|),
// compared squared), with |M(p, q)|, e^{i phi}, tau and c from the
// reciprocal square roots above.  q >= n (the dummy index of an odd order)
// or a negligible M(p, q) gives the identity.
__device__ __forceinline__ SjRot sj_rotation(int p, int q, int n, cd apq, double app, double aqq) {
    SjRot R;
    R.p = p; R.q = q; R.act = 0; R.pad = 0;
    R.c = 1.0; R.s = 0.0; R.phx = 1.0; R.phy = 0.0; R.dp = app; R.dq = aqq;
    if (q >= n) return R;
    const double eps = 2.220446049250313e-16;
    const double r2 = cabs2(apq);
    if (!(r2 > 0.0 && r2 > eps * eps * fabs(app) * fabs(aqq))) return R;
    const double ir = sj_rsqrt(r2), rr = r2 * ir;
    const double tau = 0.5 * (aqq - app) * ir, at = fabs(tau);
    // |tau| + sqrt(1 + tau^2), without overflow for huge |tau|
    double den;
    if (at > 1e150) {
        den = 2.0 * at;
    } else {
        const double u = fma(tau, tau, 1.0);
        den = at + u * sj_rsqrt(u);
    }
    const double tt = tau >= 0.0 ? sj_rcp(den) : -sj_rcp(den);
    const double c = sj_rsqrt(fma(tt, tt, 1.0));
    R.act = 1;
    R.c = c;
    R.s = tt * c;
    R.phx = apq.x * ir;
    R.phy = apq.y * ir;
    R.dp = app - tt * rr;
    R.dq = aqq + tt * rr;
    return R;
}

// Coefficients of one output of a pair's 2x2 factor: row a of U^H,
// (u0, u1) with new_a = u0 x_p + u1 x_q, is (c, -s ph) or (s, c ph); column
// b of U takes conj(ph).  Identity for a pair that does not rotate.
__device__ __forceinline__ void sj_coef(const SjRot &R, int a, bool conj_ph, double &u0, cd &u1) {
    if (!R.act) {
        u0 = a ? 0.0 : 1.0;
        u1 = cmk(a ? 1.0 : 0.0, 0.0);
        return;
    }
    const double py = conj_ph ? -R.phy : R.phy;
    u0 = a ? R.s : R.c;
    const double f = a ? R.c : -R.s;
    u1 = cmk(f * R.phx, f * py);
}

// rows (a0, a1) -> (c a0 - s ph a1, s a0 + c ph a1): the left factor U^H of a
// pair; columns use conj(ph) (the right factor U).
__device__ __forceinline__ void sj_apply(const SjRot &R, bool conj_ph, cd &a0, cd &a1) {
    const cd ph = cmk(R.phx, conj_ph ? -R.phy : R.phy);
    const cd b = cmul(ph, a1);
    const cd n0 = cmk(R.c * a0.x - R.s * b.x, R.c * a0.y - R.s * b.y);
    const cd n1 = cmk(R.s * a0.x + R.c * b.x, R.s * a0.y + R.c * b.y);
    a0 = n0;
    a1 = n1;
}

// One step for entry e = (ea, eb) of block (k1, k2), orders <= 16 (four
// threads per block, in one wave, so every read of the block precedes the
// writes: each written value depends on all four reads).  Returns the
// entry's |M(i, j)|^2 (i != j) on the last step of a sweep.
__device__ __forceinline__ double sj_entry_step(SmallLds32 &S, int n, int k1, int k2, int e, int buf, int rn,
                                                int sweep, bool last) {
    const SjRot P1 = S.rot[buf][k1], P2 = S.rot[buf][k2];
    const int ea = e >> 1, eb = e & 1;
    const int i0 = P1.p, i1 = P1.q, j0 = P2.p, j1 = P2.q;
    const int i = ea ? i1 : i0, j = eb ? j1 : j0;
    const bool r1 = i1 < n, c1 = j1 < n;  // i0, j0 < n always (p < q)
    double off = 0.0;
    cd anew = cmk(0.0, 0.0);
    if (i < n && j < n) {
        double g0;
        cd g1;
        sj_coef(P2, eb, true, g0, g1);
        if (k1 == k2) {
            anew = S.A[i + j * SJ_LD];
            if (P1.act) anew = cmk(ea == eb ? (ea ? P1.dq : P1.dp) : 0.0, 0.0);
        } else {
            const cd b00 = S.A[i0 + j0 * SJ_LD];
            const cd b01 = c1 ? S.A[i0 + j1 * SJ_LD] : cmk(0.0, 0.0);
            const cd b10 = r1 ? S.A[i1 + j0 * SJ_LD] : cmk(0.0, 0.0);
            const cd b11 = r1 && c1 ? S.A[i1 + j1 * SJ_LD] : cmk(0.0, 0.0);
            double h0;
            cd h1;
            sj_coef(P1, ea, false, h0, h1);
            // row ea of U^H B, then its column eb of (U^H B) U
            const cd t0 = cfma(h1, b10, cscale(b00, h0));
            const cd t1 = cfma(h1, b11, cscale(b01, h0));
            anew = cfma(g1, t1, cscale(t0, g0));
        }
        const cd v0 = S.V[i + j0 * SJ_LD];
        const cd v1 = c1 ? S.V[i + j1 * SJ_LD] : cmk(0.0, 0.0);
        S.A[i + j * SJ_LD] = anew;
        S.V[i + j * SJ_LD] = cfma(g1, v1, cscale(v0, g0));
        if (last && i != j) off = cabs2(anew);
    }
    if (k1 == k2 && e == 0 && P1.act) S.rotated[sweep % 3] = 1;  // benign race: all writers store 1
    // the rotation of the next step whose off-diagonal entry this is
    if (i < j && S.partner[rn][i] == j) {
        const double dii = ea ? P1.dq : P1.dp, djj = eb ? P2.dq : P2.dp;
        S.rot[buf ^ 1][S.pairof[rn][i]] = sj_rotation(i, j, n, anew, dii, j < n ? djj : 0.0);
    }
    return off;
}

// One step for the whole block (k1, k2), orders 17 .. 32: both sides of
// the two rotations on M's block, the right side on V's, then the next
// step's rotations whose entries lie here (one at most for these orders).
__device__ __forceinline__ double sj_block_step(SmallLds32 &S, int n, int k1, int k2, int buf, int rn, int sweep,
                                                bool last) {
    const SjRot P1 = S.rot[buf][k1], P2 = S.rot[buf][k2];
    const int i0 = P1.p, i1 = P1.q, j0 = P2.p, j1 = P2.q;
    const bool r1 = i1 < n, c1 = j1 < n;  // i0, j0 < n always (p < q)
    cd a00 = S.A[i0 + j0 * SJ_LD];
    cd a01 = c1 ? S.A[i0 + j1 * SJ_LD] : cmk(0.0, 0.0);
    cd a10 = r1 ? S.A[i1 + j0 * SJ_LD] : cmk(0.0, 0.0);
    cd a11 = r1 && c1 ? S.A[i1 + j1 * SJ_LD] : cmk(0.0, 0.0);
    cd v00 = S.V[i0 + j0 * SJ_LD];
    cd v01 = c1 ? S.V[i0 + j1 * SJ_LD] : cmk(0.0, 0.0);
    cd v10 = r1 ? S.V[i1 + j0 * SJ_LD] : cmk(0.0, 0.0);
    cd v11 = r1 && c1 ? S.V[i1 + j1 * SJ_LD] : cmk(0.0, 0.0);
    if (k1 == k2) {
        if (P1.act) {
            a00 = cmk(P1.dp, 0.0);
            a11 = cmk(P1.dq, 0.0);
            a01 = a10 = cmk(0.0, 0.0);
        }
    } else {
        if (P1.act) { sj_apply(P1, false, a00, a10); sj_apply(P1, false, a01, a11); }
        if (P2.act) { sj_apply(P2, true, a00, a01); sj_apply(P2, true, a10, a11); }
    }
    if (P2.act) { sj_apply(P2, true, v00, v01); sj_apply(P2, true, v10, v11); }
    S.A[i0 + j0 * SJ_LD] = a00;
    S.V[i0 + j0 * SJ_LD] = v00;
    if (c1) { S.A[i0 + j1 * SJ_LD] = a01; S.V[i0 + j1 * SJ_LD] = v01; }
    if (r1) { S.A[i1 + j0 * SJ_LD] = a10; S.V[i1 + j0 * SJ_LD] = v10; }
    if (r1 && c1) { S.A[i1 + j1 * SJ_LD] = a11; S.V[i1 + j1 * SJ_LD] = v11; }
    if (k1 == k2 && P1.act) S.rotated[sweep % 3] = 1;  // benign race: all writers store 1
    int e = -1;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const int i = (f >> 1) ? i1 : i0, j = (f & 1) ? j1 : j0;
        if (i < j && S.partner[rn][i] == j) e = f;
    }
    if (e >= 0) {
        const int i = (e >> 1) ? i1 : i0, j = (e & 1) ? j1 : j0;
        const cd aij = e == 0 ? a00 : e == 1 ? a01 : e == 2 ? a10 : a11;
        const double dii = (e >> 1) ? P1.dq : P1.dp, djj = (e & 1) ? P2.dq : P2.dp;
        S.rot[buf ^ 1][S.pairof[rn][i]] = sj_rotation(i, j, n, aij, dii, j < n ? djj : 0.0);
    }
    if (!last) return 0.0;
    return k1 != k2 ? cabs2(a00) + cabs2(a01) + cabs2(a10) + cabs2(a11) : cabs2(a01) + cabs2(a10);
}

__global__ void __launch_bounds__(SJ_NT)
small32_project_kernel(const SmallJob *jobs, SmallJob single, const double *__restrict__ xall,
                       double *yall, psd_dev_info *infos, double *saved_all) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    SmallLds32 &S = *reinterpret_cast<SmallLds32 *>(lds_raw);
    const SmallJob job = jobs ? jobs[blockIdx.x] : single;
    const int n = job.n;
    const double *x = xall + job.offset;
    double *y = yall + job.offset;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, nt = (int)blockDim.x;
    if (!small_unpack<SJ_LD>(S, job, x, y, infos)) return;

    const int m = n + (n & 1);  // an odd order gets a dummy index n that never rotates
    const int np = m / 2, R = m - 1;
    // the schedule: step r pairs r with m - 1 (pair 0) and a = r + k with
    // b = r - k mod m - 1 (pair k), so the partner of i != r is 2r - i
    for (int idx = t; idx < R * m; idx += nt) {
        const int r = idx / m, i = idx - r * m;
        int pt, k;
        if (i == m - 1 || i == r) {
            pt = i == r ? m - 1 : r;
            k = 0;
        } else {
            pt = ((2 * r - i) % R + R) % R;
            const int d = ((i - r) % R + R) % R;
            k = d <= (m - 2) / 2 ? d : R - d;
        }
        S.partner[r][i] = (unsigned char)pt;
        S.pairof[r][i] = (unsigned char)k;
    }
    // ||X||_F^2 (invariant under the rotations)
    double f2 = 0.0;
    for (int idx = t; idx < n * n; idx += nt) {
        const int i = idx % n, j = idx / n;
        f2 += cabs2(S.A[i + j * SJ_LD]);
    }
    const double nrm2 = block_sum(f2, &S.red[0][0]);
    // rotations of the first step
    if (t < np) {
        int p, q;
        rr_pair(m, 0, t, p, q);
        const cd apq = q < n ? S.A[p + q * SJ_LD] : cmk(0.0, 0.0);
        const double app = S.A[p + p * SJ_LD].x, aqq = q < n ? S.A[q + q * SJ_LD].x : 0.0;
        S.rot[0][t] = sj_rotation(p, q, n, apq, app, aqq);
    }
    if (t < 3) S.rotated[t] = 0;
    __syncthreads();

    // Orders <= 16: thread t computes entry (t / 2 % 2, t % 2) of block
    // (k1, k2) = t / 4; above, one thread per block computes all four (more
    // waves cost more at every barrier than they save).
    const bool quad = np <= 8;
    const bool worker = t < (quad ? 4 : 1) * np * np;
    const int blk = quad ? t >> 2 : t, e0 = quad ? t & 3 : 0;
    const int k1 = worker ? blk / np : 0, k2 = worker ? blk - k1 * np : 0;
    const double tol2 = SJ_TOL * SJ_TOL * nrm2;
    int buf = 0, sweep = 0;
    bool done = m < 2;  // order 0: nothing to rotate
    for (; sweep < SB_SWEEPS && !done; ++sweep) {
        if (t == 0) S.rotated[(sweep + 1) % 3] = 0;  // last read two sweeps ago
        for (int r = 0; r < R; ++r) {
            const int rn = r + 1 < R ? r + 1 : 0;
            const bool last = r == R - 1;
            double off = 0.0;
            if (worker) {
                if (quad) off = sj_entry_step(S, n, k1, k2, e0, buf, rn, sweep, last);
                else off = sj_block_step(S, n, k1, k2, buf, rn, sweep, last);
            }
            if (last) {
                off = warp_sum(off);
                if (lane == 0) S.red[sweep & 1][w] = off;
            }
            __syncthreads();
            buf ^= 1;
            if (last) {
                double o2 = 0.0;
                for (int q = 0; q < nt / 64; ++q) o2 += S.red[sweep & 1][q];
                done = o2 <= tol2 || !S.rotated[sweep % 3];
            }
        }
    }
    if (t == 0 && !done && S.status == ST_OK) S.status = ST_ENOCONV;
    __syncthreads();
    small_finish<SJ_LD>(S, job, x, y, infos, saved_all);
}

size_t small_lds_bytes() { return sizeof(SmallLds); }

static hipError_t small_attr() {
    static bool attr_set = false;
    if (attr_set) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void *)small_project_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(SmallLds));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)small32_project_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sizeof(SmallLds32));
    if (e == hipSuccess) attr_set = true;
    return e;
}

hipError_t small_prepare() { return small_attr(); }

int small32_threads(int n) { return sj_threads(n); }

hipError_t launch_small(const SmallJob *jobs, int njobs, int n32, int nt32, const double *x, double *y,
                        psd_dev_info *infos, double *saved, hipStream_t st) {
    hipError_t e = small_attr();
    if (e != hipSuccess) return e;
    SmallJob none{0, 0, 0, 0};
    if (n32 > 0)
        hipLaunchKernelGGL(small32_project_kernel, dim3(n32), dim3(nt32), sizeof(SmallLds32), st, jobs,
                           none, x, y, infos, saved);
    if (njobs > n32)
        hipLaunchKernelGGL(small_project_kernel, dim3(njobs - n32), dim3(SB_NT), sizeof(SmallLds), st, jobs + n32,
                           none, x, y, infos, saved);
    return hipGetLastError();
}

hipError_t launch_small_one(const SmallJob &job, const double *x, double *y, psd_dev_info *info,
                            double *saved, hipStream_t st) {
    hipError_t e = small_attr();
    if (e != hipSuccess) return e;
    if (job.n <= SJ_MAX)
        hipLaunchKernelGGL(small32_project_kernel, dim3(1), dim3(sj_threads(job.n)), sizeof(SmallLds32), st,
                           (const SmallJob *)nullptr, job, x, y, info, saved);
    else
        hipLaunchKernelGGL(small_project_kernel, dim3(1), dim3(SB_NT), sizeof(SmallLds), st,
                           (const SmallJob *)nullptr, job, x, y, info, saved);
    return hipGetLastError();
}

}  // namespace psd
