// Whole-block projection of small Hermitian blocks (order n <= 64) by one
// workgroup entirely in LDS.  Serves single blocks of order <= 64 (e.g. the
// d=2 process matrix, n=16) and the instrument Choi blocks (d^2 x d^2) of a
// batched cone.
//
// Steps, all in LDS (M = conj X, column-major, see common.h):
//   1. unpack the svec block (App. D.1 vec_R) into the full Hermitian M;
//   2. Householder reduction M = Q T Q^H to a real symmetric tridiagonal T
//      (reflectors H_j = I - tau_j v_j v_j^H with real subdiagonal beta_j);
//   3. implicit-shift QL iteration on T, accumulating the rotations into Z
//      (T = Z diag(lambda) Z^T);
//   4. back-transform V = Q Z for the smaller sign side only;
//   5. Pi = V+ diag(lambda+) V+^H, or X + V- diag(|lambda-|) V-^H when fewer
//      eigenvalues are non-positive (App. D.2: eigendecompose, zero the
//      negative eigenvalues), written straight back as svec.
#include "common.h"
#include "kernels.h"
#include "ql.h"

namespace psd {

constexpr int SB_MAX = 64;   // largest order served
constexpr int SB_LD = 64;    // LDS leading dimension
constexpr int SB_NT = 256;   // threads per workgroup
constexpr int SB_KMAX = 32;  // max columns back-transformed at once

struct SmallLds {
    cd A[SB_LD * SB_MAX];       // M, then reflectors below the subdiagonal
    double Z[SB_LD * SB_MAX];   // tridiagonal eigenvectors
    cd Vs[SB_LD * SB_KMAX];     // back-transformed columns
    cd part[4 * SB_MAX];        // partial row sums
    cd w[SB_MAX];
    cd tau[SB_MAX];
    double d[SB_MAX], e[SB_MAX], lam[SB_MAX];
    double rc[SB_MAX], rs[SB_MAX];
    double scal[SB_KMAX];
    int perm[SB_MAX];
    int sel[SB_KMAX];
    double red[SB_NT / 64 * 2];
    int nrot, done, status, ksel, sgn;
};

__device__ void small_ql(SmallLds &S, int n) {
    int st = ql_implicit(S.d, S.e, S.Z, SB_LD, n, S.rc, S.rs, S.perm, &S.nrot, &S.done);
    if (threadIdx.x == 0 && st != ST_OK && S.status == ST_OK) S.status = st;
    __syncthreads();
}

// Householder reduction of the Hermitian matrix in S.A (order n) to real
// tridiagonal form (d, e), reflectors stored below the diagonal with the unit
// leading entry written explicitly.
__device__ void small_tridiag(SmallLds &S, int n) {
    const int t = threadIdx.x;
    for (int j = 0; j + 1 < n; ++j) {
        const int m = n - j - 1;  // trailing order
        // sigma = sum |x_r|^2 for r >= j+2
        double part = 0.0;
        for (int r = j + 2 + t; r < n; r += SB_NT) part += cabs2(S.A[r + j * SB_LD]);
        const double sigma = block_sum(part, S.red);
        const cd alpha = S.A[(j + 1) + j * SB_LD];
        cd tau, scale;
        double beta;
        if (sigma == 0.0 && alpha.y == 0.0) {
            tau = cmk(0.0, 0.0); beta = alpha.x; scale = cmk(0.0, 0.0);
        } else {
            beta = -copysign(sqrt(cabs2(alpha) + sigma), alpha.x);
            tau = cmk((beta - alpha.x) / beta, -alpha.y / beta);
            scale = cdiv(cmk(1.0, 0.0), cmk(alpha.x - beta, alpha.y));
        }
        __syncthreads();
        for (int r = j + 2 + t; r < n; r += SB_NT) S.A[r + j * SB_LD] = cmul(S.A[r + j * SB_LD], scale);
        if (t == 0) {
            S.A[(j + 1) + j * SB_LD] = cmk(1.0, 0.0);
            S.d[j] = S.A[j + j * SB_LD].x;
            S.e[j] = beta;
            S.tau[j] = tau;
        }
        __syncthreads();
        if (tau.x == 0.0 && tau.y == 0.0) continue;
        // w = tau * A' v  over the trailing block (rows/cols j+1..n-1)
        {
            const int r = t & 63, q = t >> 6;
            cd acc = cmk(0.0, 0.0);
            if (r < m) {
                for (int c = q; c < m; c += 4)
                    acc = cfma(S.A[(j + 1 + r) + (j + 1 + c) * SB_LD], S.A[(j + 1 + c) + j * SB_LD], acc);
            }
            S.part[q * SB_MAX + r] = acc;
        }
        __syncthreads();
        cd wv = cmk(0.0, 0.0);  // conj(w_r) v_r partial
        if (t < m) {
            cd y = cadd(cadd(S.part[t], S.part[SB_MAX + t]), cadd(S.part[2 * SB_MAX + t], S.part[3 * SB_MAX + t]));
            cd w = cmul(tau, y);
            S.w[t] = w;
            wv = cmulc(w, S.A[(j + 1 + t) + j * SB_LD]);
        }
        const double wvr = block_sum(wv.x, S.red);
        const double wvi = block_sum(wv.y, S.red + SB_NT / 64);
        // alpha2 = -1/2 tau (w^H v);  w += alpha2 v
        const cd a2 = cscale(cmul(tau, cmk(wvr, wvi)), -0.5);
        if (t < m) S.w[t] = cfma(a2, S.A[(j + 1 + t) + j * SB_LD], S.w[t]);
        __syncthreads();
        // A' -= v w^H + w v^H
        for (int idx = t; idx < m * m; idx += SB_NT) {
            const int r = idx % m, c = idx / m;
            const cd vr = S.A[(j + 1 + r) + j * SB_LD], vc = S.A[(j + 1 + c) + j * SB_LD];
            const cd wr = S.w[r], wc = S.w[c];
            cd a = S.A[(j + 1 + r) + (j + 1 + c) * SB_LD];
            a = csub(a, cmul(vr, cconj(wc)));
            a = csub(a, cmul(wr, cconj(vc)));
            S.A[(j + 1 + r) + (j + 1 + c) * SB_LD] = a;
        }
        __syncthreads();
    }
    if (t == 0) S.d[n - 1] = S.A[(n - 1) + (n - 1) * SB_LD].x;
    __syncthreads();
}

// Vs[:, 0:k] = Q Z[:, cols] with Q = H_0 H_1 ... H_{n-2}; cols given by
// column indices colidx[0..k) of Z.  k <= SB_KMAX.
__device__ void small_backtransform(SmallLds &S, int n, int k, const int *colidx) {
    const int t = threadIdx.x;
    for (int idx = t; idx < n * k; idx += SB_NT) {
        const int r = idx % n, c = idx / n;
        S.Vs[r + c * SB_LD] = cmk(S.Z[r + colidx[c] * SB_LD], 0.0);
    }
    __syncthreads();
    // 8 lanes per column: lane group g = t/8 handles column g (k <= 32)
    const int c = t >> 3, sub = t & 7;
    for (int j = n - 2; j >= 0; --j) {
        const cd tj = S.tau[j];
        if (tj.x == 0.0 && tj.y == 0.0) continue;  // uniform across the block
        cd acc = cmk(0.0, 0.0);
        if (c < k)
            for (int r = j + 1 + sub; r < n; r += 8) acc = cfmac(S.A[r + j * SB_LD], S.Vs[r + c * SB_LD], acc);
#pragma unroll
        for (int o = 1; o < 8; o <<= 1) {
            acc.x += __shfl_xor(acc.x, o, 64);
            acc.y += __shfl_xor(acc.y, o, 64);
        }
        const cd f = cmul(tj, acc);
        if (c < k)
            for (int r = j + 1 + sub; r < n; r += 8)
                S.Vs[r + c * SB_LD] = csub(S.Vs[r + c * SB_LD], cmul(S.A[r + j * SB_LD], f));
        __syncthreads();
    }
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
        S.Z[i + j * SB_LD] = (i == j) ? 1.0 : 0.0;
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

    // 2-3. tridiagonalise, then QL
    small_tridiag(S, n);
    small_ql(S, n);

    // ascending order of the eigenvalues
    if (t < n) {
        const double v = S.d[t];
        int rank = 0;
        for (int q = 0; q < n; ++q) {
            const double u = S.d[q];
            rank += (u < v) || (u == v && q < t);
        }
        S.lam[rank] = v;
        S.perm[rank] = t;  // column of Z
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

    // optional: full eigenvectors for a later derivative
    if (saved_all) {
        double *sv = saved_all + job.saved_offset;
        if (t < n) sv[t] = S.lam[t];
        cd *V = reinterpret_cast<cd *>(sv + n);
        for (int c0 = 0; c0 < n; c0 += SB_KMAX) {
            const int kc = min(SB_KMAX, n - c0);
            small_backtransform(S, n, kc, S.perm + c0);
            for (int idx = t; idx < n * kc; idx += SB_NT) {
                const int r = idx % n, c = idx / n;
                V[r + (long)(c0 + c) * n] = S.Vs[r + c * SB_LD];
            }
            __syncthreads();
        }
    }

    // 4. back-transform the selected side
    const int k = S.ksel;
    small_backtransform(S, n, k, S.sel);

    // 5. reconstruct the lower triangle and pack.  Each thread reads x and
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
        for (int c = 0; c < k; ++c)
            acc = cfma(cscale(S.Vs[i + c * SB_LD], S.scal[c]), cconj(S.Vs[j + c * SB_LD]), acc);
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
