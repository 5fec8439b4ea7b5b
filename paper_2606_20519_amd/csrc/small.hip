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
// its rotations one after another.
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

__global__ void __launch_bounds__(SB_NT)
small_project_kernel(const SmallJob *jobs, SmallJob single, const double *__restrict__ xall,
                     double *yall, psd_dev_info *infos, double *saved_all) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    SmallLds &S = *reinterpret_cast<SmallLds *>(lds_raw);
    const SmallJob job = jobs ? jobs[blockIdx.x] : single;
    const int n = job.n;
    const int t = threadIdx.x;
    const double *x = xall + job.offset;
    double *y = yall + job.offset;
    const double rs2 = 0.70710678118654752440;

    if (t == 0) S.status = ST_OK;
    __syncthreads();
    // 1. unpack (lower triangle of M from svec columns, mirrored)
    int bad = 0;
    for (int idx = t; idx < n * n; idx += SB_NT) {
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
        S.A[i + j * SB_LD] = v;
        S.A[j + i * SB_LD] = cconj(v);
    }
    for (int idx = t; idx < n * n; idx += SB_NT) {
        const int i = idx % n, j = idx / n;
        S.V[i + j * SB_LD] = cmk((i == j) ? 1.0 : 0.0, 0.0);
    }
    if (bad) S.status = ST_ENONFINITE;  // benign race: all writers store the same value
    __syncthreads();
    if (S.status != ST_OK) {
        // Non-finite input: the projection is undefined; report it and
        // return NaN in every entry.
        for (int idx = t; idx < n * n; idx += SB_NT) {
            const int i = idx % n, j = idx / n;
            if (i < j) continue;
            if (i == j) y[svec_col_start(n, j)] = __builtin_nan("");
            else { const long o = svec_off(n, i, j); y[o] = __builtin_nan(""); y[o + 1] = __builtin_nan(""); }
        }
        if (t == 0 && infos) {
            psd_dev_info &I = infos[job.info_index];
            I.status = ST_ENONFINITE; I.n_pos = 0; I.n_neg = 0; I.iters = 0; I.fallback = 0; I.est_rel_err = 0.0; I.scale = 0.0; I.scale = 0.0;
        }
        return;
    }

    // 2. Jacobi
    small_jacobi(S, n);

    // ascending order of the eigenvalues (the diagonal of the rotated M)
    if (t < n) {
        const double v = S.A[t + t * SB_LD].x;
        int rank = 0;
        for (int q = 0; q < n; ++q) {
            const double u = S.A[q + q * SB_LD].x;
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
        for (int idx = t; idx < n * n; idx += SB_NT) {
            const int r = idx % n, c = idx / n;
            V[r + (long)c * n] = S.V[r + S.perm[c] * SB_LD];
        }
    }

    const int k = S.ksel;

    // 3. reconstruct the lower triangle and pack.  Each thread reads x and
    //    writes y at the same svec positions, so y may alias x.
    //    sgn>0: Pi = sum_{lambda>0} lambda v v^H;
    //    sgn<0: Pi = X - sum_{lambda<=0} lambda v v^H.
    const int sgn = S.sgn;
    const double sd = sgn > 0 ? 1.0 : -1.0;
    const double so = sd * 1.41421356237309504880;
    for (int idx = t; idx < n * n; idx += SB_NT) {
        const int i = idx % n, j = idx / n;
        if (i < j) continue;
        cd acc = cmk(0.0, 0.0);
        for (int c = 0; c < k; ++c) {
            const int col = S.sel[c];
            acc = cfma(cscale(S.V[i + col * SB_LD], S.scal[c]), cconj(S.V[j + col * SB_LD]), acc);
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

size_t small_lds_bytes() { return sizeof(SmallLds); }

static hipError_t small_attr() {
    static bool attr_set = false;
    if (attr_set) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void *)small_project_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(SmallLds));
    if (e == hipSuccess) attr_set = true;
    return e;
}

hipError_t small_prepare() { return small_attr(); }

hipError_t launch_small(const SmallJob *jobs, int njobs, const double *x, double *y,
                        psd_dev_info *infos, double *saved, hipStream_t st) {
    hipError_t e = small_attr();
    if (e != hipSuccess) return e;
    SmallJob none{0, 0, 0, 0};
    hipLaunchKernelGGL(small_project_kernel, dim3(njobs), dim3(SB_NT), sizeof(SmallLds), st, jobs, none, x,
                       y, infos, saved);
    return hipGetLastError();
}

hipError_t launch_small_one(const SmallJob &job, const double *x, double *y, psd_dev_info *info,
                            double *saved, hipStream_t st) {
    hipError_t e = small_attr();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(small_project_kernel, dim3(1), dim3(SB_NT), sizeof(SmallLds), st,
                       (const SmallJob *)nullptr, job, x, y, info, saved);
    return hipGetLastError();
}

}  // namespace psd
