// FP64 projection of a block from the eigen-pair of a nearby matrix.
//
// Successive cone inputs of the splitting method differ by small steps
// (warm starting, App. D.2; the warm-started refinement stage, Sec. IV), so
// the eigenvectors V_prev of the previous input are a close approximation of
// those of the new one, A.  Instead of reducing A from scratch, the pair is
// refined by the iteration of Ogita and Aishima (Japan J. Indust. Appl.
// Math. 35, 2018), written here for complex Hermitian A; every step is three
// matrix products and one elementwise pass:
//   G = X^H X,  S = X^H (A X),  R = I - G,
//   lambda_i = S_ii / G_ii                       (Rayleigh quotients),
//   E_ii = R_ii / 2,
//   E_ij = (S_ij + lambda_j R_ij) / (lambda_j - lambda_i)   (i != j),
//   X <- X + X E.
// (The first-order conditions of (I + E)^H G (I + E) = I and
// (I + E)^H S (I + E) = diag(lambda) give E + E^H = R and, off the diagonal,
// E_ij (lambda_i - lambda_j) = -(S_ij + lambda_j R_ij).)  The error of X is
// squared by each step.  Pairs whose Rayleigh quotients agree to 2^-40 of
// the largest are treated as one cluster (E_ij = R_ij / 2, no rotation
// inside it): the projection only needs the cluster's subspace, and within
// it Pi is lambda_+ times its projector up to that spread.
//
// The result is Pi(A) = X diag(max(lambda, 0)) X^H, packed into the svec by
// the GEMM epilogue.  The iteration stops once the largest off-diagonal
// |E_ij| of a step is <= 1e-7 (the next would change X by ~1e-14) and is
// accepted when the last step's is <= 1e-6; anything else (a step limit of
// five, a basis that was not close, a non-finite input) leaves the decision
// to the host, which then runs the cold FP64 path instead.  A refinement
// that is not converging is cut short: a step above 1/2, or above half the
// previous step, skips the rest.
//
// Products run as split-K GEMMs (partials summed by the passes that read
// them) so that a block of a few hundred rows still fills the chip; every
// sum is in a fixed order, so the result is deterministic.  Steps after
// convergence are skipped on the device (the GEMMs read a flag).
#include <algorithm>

#include "common.h"
#include "gemm.h"
#include "warm.h"

namespace psd {

namespace {

constexpr int WT = 32;  // tile of the correction pass

// max that keeps a NaN from either side (fmax and a plain comparison each
// drop it from one side): a refinement that blew up must not report a
// finite step size
__device__ __forceinline__ double nanmax(double a, double b) {
    return (a != a || b != b) ? __builtin_nan("") : fmax(a, b);
}

__global__ void __launch_bounds__(64) wm_init_kernel(int *flags, int nflags) {
    for (int i = threadIdx.x; i < nflags; i += 64) flags[i] = 0;
}

// svec -> full Hermitian M = conj(X) (column-major, ld), as the cold path
// reads it; a non-finite entry sets flags[WF_STATUS].
__global__ void __launch_bounds__(256) wm_unpack_kernel(const double *__restrict__ x, double2 *A, int64_t ld, int n,
                                                        int *flags) {
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
    if (!isfinite(v.x) || !isfinite(v.y)) flags[WF_STATUS] = 1;
    A[i + (int64_t)j * ld] = v;
    if (i != j) A[j + (int64_t)i * ld] = cconj(v);
}

__global__ void __launch_bounds__(64) wm_gate_kernel(int *flags) {
    if (threadIdx.x == 0) flags[WF_SKIP] = flags[WF_STATUS];
}

// The previous eigenvectors (columns of the saved record, ld n) as X.
__global__ void __launch_bounds__(256) wm_load_kernel(const double *__restrict__ saved, int n, double2 *X,
                                                      int64_t ld) {
    const int c = blockIdx.y;
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    const double2 *V = reinterpret_cast<const double2 *>(saved + n);
    X[r + (int64_t)c * ld] = V[r + (int64_t)c * n];
}

// out = sum of the ks partials (+ add when non-null; out = add alone when
// the step is skipped).
__global__ void __launch_bounds__(256) wm_sum_kernel(const double2 *__restrict__ part, int ks, int64_t zs,
                                                     const double2 *__restrict__ add, double2 *out, int64_t ld,
                                                     int n, const int *skip) {
    const int c = blockIdx.y;
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    const int64_t idx = r + (int64_t)c * ld;
    const bool skipped = *skip != 0;
    if (skipped && !add) return;
    double2 acc = add ? add[idx] : cmk(0.0, 0.0);
    if (!skipped)
        for (int z = 0; z < ks; ++z) acc = cadd(acc, part[idx + z * zs]);
    out[idx] = acc;
}

// max |lambda| of the previous pair (one workgroup, once per call): the scale
// of the cluster threshold.
__global__ void __launch_bounds__(1024) wm_scale_kernel(const double *__restrict__ saved, int n, double *scal) {
    __shared__ double red[16];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) m = nanmax(m, fabs(saved[i]));
    for (int o = 32; o > 0; o >>= 1) m = nanmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = red[0];
        for (int w = 1; w < 16; ++w) t = nanmax(t, red[w]);
        scal[WS_LMAX] = t;
    }
}

// Rayleigh quotient Re S_kk / Re G_kk from the partials (every workgroup
// that needs index k forms it the same way, so the values agree bitwise).
__device__ __forceinline__ double wm_rayleigh(const double2 *__restrict__ pS, const double2 *__restrict__ pG, int ks,
                                              int64_t zs, int64_t ld, int k) {
    const int64_t idx = k + (int64_t)k * ld;
    double sv = 0.0, gv = 0.0;
    for (int z = 0; z < ks; ++z) {
        sv += pS[idx + z * zs].x;
        gv += pG[idx + z * zs].x;
    }
    return sv / gv;
}

// The correction E on a lower tile pair: workgroup b handles the WT x WT
// tile (I, J), I >= J, from the lower partials of S and G, and writes both
// E(I, J) and E(J, I) (the latter through LDS, so both stores run along
// columns).  The Rayleigh quotients of its rows and columns come from the
// partials' diagonals; the diagonal pairs store those of their rows in lam.
// Also the largest off-diagonal |E_ij|^2 of the pair, to epart[b].
__global__ void __launch_bounds__(256) wm_correction_kernel(const double2 *__restrict__ pS,
                                                            const double2 *__restrict__ pG, int ks, int64_t zs,
                                                            int64_t ld, int n, double *lam,
                                                            const double *__restrict__ scal, double2 *E,
                                                            double *epart, const int *skip) {
    if (*skip) return;
    __shared__ double2 U[WT][WT + 1];
    __shared__ double red[4];
    __shared__ double lr[WT], lc[WT];  // Rayleigh quotients of the pair's rows and columns
    // lower tile pair b -> (I, J), column by column
    const int nt = (n + WT - 1) / WT;
    int b = blockIdx.x, J = 0;
    while (b >= nt - J) {
        b -= nt - J;
        ++J;
    }
    const int I = J + b;
    const int t = threadIdx.x, r = t % WT, c0 = t / WT;
    if (t < 2 * WT) {
        const int k = (t < WT ? I : J) * WT + (t % WT);
        const double l = k < n ? wm_rayleigh(pS, pG, ks, zs, ld, k) : 0.0;
        if (t < WT) lr[t] = l;
        else lc[t - WT] = l;
        if (t < WT && I == J && k < n) lam[k] = l;
    }
    __syncthreads();
    const double tau = 0x1p-40 * scal[WS_LMAX];
    double emax = 0.0;
    const int i = I * WT + r;
#pragma unroll
    for (int k = 0; k < WT / 8; ++k) {
        const int c = c0 + 8 * k;
        const int j = J * WT + c;
        if (i >= n || j >= n || (I == J && r < c)) continue;
        const int64_t idx = i + (int64_t)j * ld;
        double2 s = cmk(0.0, 0.0), g = cmk(0.0, 0.0);
        for (int z = 0; z < ks; ++z) {
            s = cadd(s, pS[idx + z * zs]);
            g = cadd(g, pG[idx + z * zs]);
        }
        if (i == j) {
            E[idx] = cmk(0.5 * (1.0 - g.x), 0.0);
            continue;
        }
        const double li = lr[r], lj = lc[c];
        // E(i, j): R_ij = -G_ij
        double2 eij, eji;
        const double d = lj - li;
        if (fabs(d) > tau) {
            eij = cscale(csub(s, cscale(g, lj)), 1.0 / d);
            // E(j, i) from S_ji = conj S_ij, G_ji = conj G_ij
            eji = cscale(csub(cconj(s), cscale(cconj(g), li)), -1.0 / d);
        } else {
            eij = cscale(g, -0.5);
            eji = cscale(cconj(g), -0.5);
        }
        E[idx] = eij;
        U[c][r] = eji;
        emax = nanmax(emax, nanmax(cabs2(eij), cabs2(eji)));
    }
    __syncthreads();
    // E(J, I) = transpose of the pair's upper values: row J*WT + r, column I*WT + c
#pragma unroll
    for (int k = 0; k < WT / 8; ++k) {
        const int c = c0 + 8 * k;
        const int row = J * WT + r, col = I * WT + c;
        if (row >= n || col >= n || (I == J && r >= c)) continue;
        E[row + (int64_t)col * ld] = U[r][c];
    }
    for (int o = 32; o > 0; o >>= 1) emax = nanmax(emax, __shfl_xor(emax, o, 64));
    if ((t & 63) == 0) red[t >> 6] = emax;
    __syncthreads();
    if (t == 0) {
        double m = red[0];
        for (int w = 1; w < 4; ++w) m = nanmax(m, red[w]);
        epart[blockIdx.x] = m;
    }
}

// After step k: e = max |E_ij| over the pairs; step k + 1 is skipped once
// e <= 1e-7, when the refinement stalls (or when step k was).
__global__ void __launch_bounds__(256) wm_step_kernel(const double *__restrict__ epart, int np, double *scal,
                                                      int *flags, int k) {
    if (flags[WF_SKIP + k]) {
        if (threadIdx.x == 0) flags[WF_SKIP + k + 1] = 1;
        return;
    }
    __shared__ double red[4];
    double m = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) m = nanmax(m, epart[i]);
    for (int o = 32; o > 0; o >>= 1) m = nanmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double e2 = red[0];
        for (int w = 1; w < 4; ++w) e2 = nanmax(e2, red[w]);
        const double e = sqrt(e2);
        // stop once converged, and give up early (the host then runs the
        // cold path) when a step is not even half the previous one or
        // rotates by more than half a radian: a refinement that converges
        // squares its step
        const bool stall = e > WARM_GIVE_UP || (k > 0 && e > 0.5 * scal[WS_ELAST]);
        scal[WS_ELAST] = e;
        flags[WF_ITERS] += 1;
        flags[WF_SKIP + k + 1] = (e <= WARM_STOP || stall) ? 1 : 0;
    }
}

// Acceptance, lambda_+ for the reconstruction, counts and the info record.
__global__ void __launch_bounds__(1024) wm_final_kernel(const double *__restrict__ lam, double *lamp, int n,
                                                        const double *__restrict__ scal, int *flags,
                                                        psd_dev_info *info) {
    __shared__ int cnt[16];
    const double e = scal[WS_ELAST];
    const bool accept = flags[WF_STATUS] == 0 && flags[WF_ITERS] > 0 && e <= WARM_ACCEPT &&
                        isfinite(scal[WS_LMAX]);
    int pos = 0;
    for (int i = threadIdx.x; i < n; i += 1024) {
        const double l = lam[i];
        lamp[i] = l > 0.0 ? l : 0.0;
        pos += l > 0.0 ? 1 : 0;
    }
    for (int o = 32; o > 0; o >>= 1) pos += __shfl_xor(pos, o, 64);
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = pos;
    __syncthreads();
    if (threadIdx.x == 0) {
        int npos = 0;
        for (int w = 0; w < 16; ++w) npos += cnt[w];
        flags[WF_REJECT] = accept ? 0 : 1;
        if (info && accept) {
            info->status = 0;
            info->n_pos = npos;
            info->n_neg = n - npos;
            info->iters = flags[WF_ITERS];
            info->fallback = 0;
            info->reserved = 0;
            info->est_rel_err = e * e;
            info->scale = 0.0;
        }
    }
}

// saved_out <- (lambda, X) when the result is accepted.
__global__ void __launch_bounds__(256) wm_save_kernel(const double *__restrict__ lam, const double2 *__restrict__ X,
                                                      int64_t ld, int n, double *saved, const int *flags) {
    if (flags[WF_REJECT]) return;
    const int c = blockIdx.y;
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    if (c == 0) saved[r] = lam[r];
    double2 *V = reinterpret_cast<double2 *>(saved + n);
    V[r + (int64_t)c * n] = X[r + (int64_t)c * ld];
}

}  // namespace

// Split-K slices of a product over `tiles` output tiles: enough workgroups
// (about 512) but at most one round of them (three per CU), at most 8
// slices, each a multiple of the 16-deep k-step.
static void warm_split(int n, int tiles, int *ks, int *kchunk) {
    int s = std::min(8, std::max(1, (512 + tiles - 1) / tiles));
    s = std::max(1, std::min(s, 768 / tiles));
    const int kc = ((n + s - 1) / s + 15) / 16 * 16;
    *kchunk = kc;
    *ks = (n + kc - 1) / kc;
}

size_t warm_layout(int n, void *base, WarmWs *w) {
    size_t off = 0;
    char *b = static_cast<char *>(base);
    auto take = [&](size_t bytes) -> void * {
        void *p = b ? b + off : nullptr;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    WarmWs W{};
    W.n = n;
    W.ld = n;
    const int t = (n + 63) / 64;
    warm_split(n, t * t, &W.ksf, &W.kcf);
    warm_split(n, t * (t + 1) / 2, &W.ksl, &W.kcl);
    const int ksmax = std::max(W.ksf, W.ksl);
    const size_t mat = sizeof(double2) * (size_t)n * (size_t)n;
    W.A = static_cast<double2 *>(take(mat));
    W.X[0] = static_cast<double2 *>(take(mat));
    W.X[1] = static_cast<double2 *>(take(mat));
    W.B = static_cast<double2 *>(take(mat));
    W.E = static_cast<double2 *>(take(mat));
    W.P1 = static_cast<double2 *>(take(mat * ksmax));
    W.P2 = static_cast<double2 *>(take(mat * W.ksl));
    W.lam = static_cast<double *>(take(sizeof(double) * n));
    W.lamp = static_cast<double *>(take(sizeof(double) * n));
    const int nt = (n + WT - 1) / WT;
    W.npairs = nt * (nt + 1) / 2;
    W.epart = static_cast<double *>(take(sizeof(double) * W.npairs));
    W.scal = static_cast<double *>(take(sizeof(double) * 4));
    W.flags = static_cast<int *>(take(sizeof(int) * WF_COUNT));
    if (w) *w = W;
    return off;
}

hipError_t warm_refine(const WarmWs &w, const double *x, const double *saved_prev, double *y, double *saved_out,
                       psd_dev_info *info, hipStream_t st) {
    const int n = w.n;
    const int64_t ld = w.ld, zs = (int64_t)n * ld;
    const dim3 gcol((n + 255) / 256, n);
    hipLaunchKernelGGL(wm_init_kernel, dim3(1), dim3(64), 0, st, w.flags, (int)WF_COUNT);
    hipLaunchKernelGGL(wm_unpack_kernel, gcol, dim3(256), 0, st, x, w.A, ld, n, w.flags);
    hipLaunchKernelGGL(wm_load_kernel, gcol, dim3(256), 0, st, saved_prev, n, w.X[0], ld);
    hipLaunchKernelGGL(wm_scale_kernel, dim3(1), dim3(1024), 0, st, saved_prev, n, w.scal);
    // a non-finite input skips every step (the host then runs the cold path)
    hipLaunchKernelGGL(wm_gate_kernel, dim3(1), dim3(64), 0, st, w.flags);
    auto product = [&](const double2 *a, int opa, const double2 *bm, int opb, int lower, const int *skip) {
        GemmDesc g{};
        g.kchunk = lower ? w.kcl : w.kcf;
        g.M = g.N = g.K = n;
        g.lower_only = lower;
        g.A = GemmOperand{a, a, ld, ld, n, opa, nullptr};
        g.B = GemmOperand{bm, bm, ld, ld, n, opb, nullptr};
        g.ldc = ld;
        g.alpha = 1.0;
        g.beta = 0.0;
        g.c_zstride = zs;
        g.skip = skip;
        return g;
    };
    hipError_t e;
    for (int k = 0; k < WARM_STEPS; ++k) {
        const double2 *X = w.X[k & 1];
        double2 *Xn = w.X[(k + 1) & 1];
        const int *skip = w.flags + WF_SKIP + k;
        // B = A X
        GemmDesc g = product(w.A, OP_N, X, OP_N, 0, skip);
        g.C = w.P1;
        if ((e = gemm_launch(g, true, EPI_STORE, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(wm_sum_kernel, gcol, dim3(256), 0, st, w.P1, w.ksf, zs, nullptr, w.B, ld, n, skip);
        // S = X^H B and G = X^H X, lower tiles (summed by the passes below)
        g = product(X, OP_C, w.B, OP_N, 1, skip);
        g.C = w.P1;
        if ((e = gemm_launch(g, true, EPI_STORE, st)) != hipSuccess) return e;
        g = product(X, OP_C, X, OP_N, 1, skip);
        g.C = w.P2;
        if ((e = gemm_launch(g, true, EPI_STORE, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(wm_correction_kernel, dim3(w.npairs), dim3(256), 0, st, w.P1, w.P2, w.ksl, zs, ld, n,
                           w.lam, w.scal, w.E, w.epart, skip);
        hipLaunchKernelGGL(wm_step_kernel, dim3(1), dim3(256), 0, st, w.epart, w.npairs, w.scal, w.flags, k);
        // X_next = X + X E (a copy of X when the step is skipped)
        g = product(X, OP_N, w.E, OP_N, 0, skip);
        g.C = w.P1;
        if ((e = gemm_launch(g, true, EPI_STORE, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(wm_sum_kernel, gcol, dim3(256), 0, st, w.P1, w.ksf, zs, X, Xn, ld, n, skip);
    }
    const double2 *Xf = w.X[WARM_STEPS & 1];
    hipLaunchKernelGGL(wm_final_kernel, dim3(1), dim3(1024), 0, st, w.lam, w.lamp, n, w.scal, w.flags, info);
    // y = svec(X diag(lambda_+) X^H), lower tiles, unless rejected
    GemmDesc r{};
    r.M = r.N = r.K = n;
    r.lower_only = 1;
    r.A = GemmOperand{Xf, Xf, ld, ld, n, OP_N, w.lamp};
    r.B = GemmOperand{Xf, Xf, ld, ld, n, OP_C, nullptr};
    r.y = y;
    r.svec_n = n;
    r.sign = 1.0;
    r.skip = w.flags + WF_REJECT;
    if ((e = gemm_launch(r, true, EPI_SVEC, st)) != hipSuccess) return e;
    if (saved_out) hipLaunchKernelGGL(wm_save_kernel, gcol, dim3(256), 0, st, w.lam, Xf, ld, n, saved_out, w.flags);
    return hipGetLastError();
}

}  // namespace psd
