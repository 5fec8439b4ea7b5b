// SCS iteration for the bipartite process-matrix SDP on the GPU (App. D):
//
//     min c^T x  s.t.  A x + s = b,  s in H_+^{d^4},
//
// with A x = -sum_mu x_mu F_mu over the allowed multi-indices, b = gamma 1
// (gamma = 1/d^2) and c = A^T G for the game objective G (c_mu = -tr[G F_mu],
// eq. constraint_map_def), solved through the homogeneous self-dual embedding
// by the splitting iteration of eq. final_iterates
//
//     u~ = (1 + Q)^-1 (u + v),   u = Pi_C(u~_r - v),   v = v - u~_r + u,
//
// u = (x, y, tau), v = (r, s, kappa), C = R^n x H_+ x R_+, with the
// over-relaxed u~_r = alpha u~ + (1 - alpha) u.  Every vector lives in device
// memory for the whole solve; each step is a kernel:
//
//  * (1 + Q)^-1 by the Sherman-Morrison form of App. D.1 ("Solving the affine
//    projection"): with h = (c, b) and M = [[1, A^T], [-A, 1]],
//    u~_xy = z - u~_tau M^-1 h and u~_tau = a_tau + (h^T z - a_tau eta) /
//    (1 + eta), z = M^-1 a_xy, eta = h^T M^-1 h -- the same vector as the
//    printed rank-one update, in a form that needs one dot product h^T z per
//    iteration (h^T u~_xy = (h^T z - a_tau eta)/(1 + eta) because
//    h^T w (1 - eta/(1 + eta)) = h^T w / (1 + eta)).  M^-1 is the closed form
//    of psd_affine_step (A^T A = I).  b^T z_y only reads the n diagonal
//    entries of z_y.
//  * Pi_C: x free, y by psd_project (the PSD cone, in place), tau clamped at
//    0 by a one-thread kernel that also keeps kappa.  r = v_x stays 0: the
//    cone's first factor is all of R^n, so v_x = v_x - u~_x + u~_x - v_x.
//  * the iterate is fixed by the cone step's input q = u~_r - v alone
//    (u = Pi_C(q) and v = u - q, Moreau), kept as (u_x, the svec z_y, a
//    device scalar): the cone step projects z_y into u_y and sets
//    v_s = u_y - z_y, tau = max(q_tau, 0), kappa = tau - q_tau.
//  * type-I Anderson acceleration (optional, memory m <= 16) of the map
//    q -> G(q) (cone step, then affine step): the m last differences of q and
//    of f = q - G(q) live in HBM; one fused pass writes the new pair, one
//    computes all the new inner products (block partials, then one block per
//    product), the host solves the m x m system (S^T Y + lam 1) gamma = S^T f
//    (lam = 1e-8 ||S||_F ||Y||_F), and one pass forms G(q) - (S - Y) gamma.
//    Safeguard: an accelerated input whose residual exceeds twice the
//    previous one is replaced by the plain G(q) it displaced and the memory
//    is cleared; |gamma| > 1e10 or a singular system skips the step.
//  * the termination test of App. D.1 ("Convergence criteria") on
//    x = u_x / tau, s = v_s / tau and y = u_y / (sigma tau) (sigma: partial
//    normalisation, App. D.2), eps_abs = eps_rel = eps, evaluated every
//    `check_every` iterations from one A u_x, one A^T u_y and deterministic
//    two-level reductions read back by the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/psdproj.h"
#include "affine.h"
#include "common.h"

namespace psd {

namespace {

static_assert(sizeof(psd_scs_settings) == 64, "psd_scs_settings layout");
static_assert(sizeof(psd_scs_info) == 112, "psd_scs_info layout");

constexpr int SCS_BLOCK = 256;
constexpr int SCS_PARTS = 512;   // blocks of the first reduction level

// Device scalars of the iteration.
enum { SC_UT = 0, SC_VK = 1, SC_UTT = 2, SC_QT = 3, SC_SIGMA = 4, SC_ETA = 5, SC_COUNT = 8 };

// Instance blockIdx.z of a batch: its slot vectors sit `slot` bytes apart,
// its cone-step blocks (u_y, z_y) `blk` bytes apart; `active` (nullable)
// marks the instances still running (the others are left untouched).
struct ScsZ {
    int64_t slot, blk;
    const int *active;
};
template <class T>
__device__ __forceinline__ T *zmove(T *p, int64_t bytes) {
    return reinterpret_cast<T *>(reinterpret_cast<uintptr_t>(p) + (uintptr_t)(bytes * (int64_t)blockIdx.z));
}
__device__ __forceinline__ bool zrunning(const ScsZ &z) { return !z.active || z.active[blockIdx.z]; }
// Reduction slots.
enum {
    R_PRI = 0,     // max |A u_x + v_s - tau b|
    R_AX = 1,      // max |A u_x|
    R_S = 2,       // max |v_s|
    R_DUAL = 3,    // max |A^T u_y + sigma tau c|
    R_ATY = 4,     // max |A^T u_y|
    R_CX = 5,      // sum c_i u_x,i
    R_TRY = 6,     // sum of the diagonal of u_y
    R_SLOTS = 7
};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

__device__ __forceinline__ double nan_max(double m, double v) { return (v > m || v != v) ? v : m; }

// Block-wide reduction of `nv` values per thread (sums or NaN-propagating
// maxima), written to part[slot * SCS_PARTS + blockIdx.x].
template <int NV>
__device__ void block_reduce(double (&v)[NV], const bool (&is_max)[NV], const int (&slot)[NV], double *part) {
    __shared__ double red[NV][SCS_BLOCK / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double y = __shfl_xor(x, o, 64);
            x = is_max[k] ? nan_max(x, y) : x + y;
        }
        if (lane == 0) red[k][w] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double x = red[k][0];
            for (int q = 1; q < SCS_BLOCK / 64; ++q) x = is_max[k] ? nan_max(x, red[k][q]) : x + red[k][q];
            part[slot[k] * SCS_PARTS + blockIdx.x] = x;
        }
    }
}

// a = u + v (v_x = 0): z_x = u_x, z_y = u_y + v_s.
__global__ void __launch_bounds__(SCS_BLOCK) scs_sum_kernel(const double *__restrict__ ux, const double *__restrict__ uy,
                                                            const double *__restrict__ vy, double *zx, double *zy,
                                                            int64_t nx, int64_t ny, ScsZ z) {
    if (!zrunning(z)) return;
    ux = zmove(ux, z.slot); vy = zmove(vy, z.slot); zx = zmove(zx, z.slot);
    uy = zmove(uy, z.blk); zy = zmove(zy, z.blk);
    const int64_t t = (int64_t)blockIdx.x * SCS_BLOCK + threadIdx.x;
    if (t < nx) zx[t] = ux[t];
    else if (t < nx + ny) zy[t - nx] = uy[t - nx] + vy[t - nx];
}

// Partial sums of h^T z = sigma c^T z_x + gamma tr(z_y) into part[0 ..)
// (sigma = sc[SC_SIGMA]).
__global__ void __launch_bounds__(SCS_BLOCK) scs_dot_kernel(const double *__restrict__ c,
                                                            const double *__restrict__ zx,
                                                            const double *__restrict__ zy, int64_t nx, int n,
                                                            const double *__restrict__ sc, double gamma, double *part,
                                                            ScsZ z) {
    if (!zrunning(z)) return;
    c = zmove(c, z.slot); zx = zmove(zx, z.slot); sc = zmove(sc, z.slot); part = zmove(part, z.slot);
    zy = zmove(zy, z.blk);
    const double sigma = sc[SC_SIGMA];
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * SCS_BLOCK + threadIdx.x; t < nx + n; t += (int64_t)gridDim.x * SCS_BLOCK)
        acc += t < nx ? sigma * c[t] * zx[t] : gamma * zy[svec_col_start(n, (int)(t - nx))];
    double v[1] = {acc};
    const bool mx[1] = {false};
    const int sl[1] = {0};
    block_reduce<1>(v, mx, sl, part);
}

// Sum of the first `parts` partials of each of `nslots` slots, in a fixed
// order (one wave per slot).
__device__ double sum_parts(const double *part, int slot, int parts, bool is_max) {
    const int lane = threadIdx.x & 63;
    double x = 0.0;   // the maxima are of absolute values
    for (int q = lane; q < parts; q += 64) x = is_max ? nan_max(x, part[slot * SCS_PARTS + q]) : x + part[slot * SCS_PARTS + q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double y = __shfl_xor(x, o, 64);
        x = is_max ? nan_max(x, y) : x + y;
    }
    return x;
}

// tau part of the affine step: u~_tau, then the cone input
// q_tau = alpha u~_tau + (1 - alpha) tau - kappa.  One wave.
__global__ void __launch_bounds__(64) scs_tau_kernel(const double *part, int parts, double *sc, double alpha,
                                                     ScsZ z) {
    if (!zrunning(z)) return;
    part = zmove(part, z.slot); sc = zmove(sc, z.slot);
    const double hz = sum_parts(part, 0, parts, false);
    if (threadIdx.x != 0) return;
    const double eta = sc[SC_ETA];
    const double ut = sc[SC_UT], vk = sc[SC_VK];
    const double at = ut + vk;
    const double utt = at + (hz - at * eta) / (1.0 + eta);
    sc[SC_UTT] = utt;
    sc[SC_QT] = alpha * utt + (1.0 - alpha) * ut - vk;
}

// u~_xy = z - u~_tau M^-1 h; relaxed r = alpha u~ + (1 - alpha) u; the cone
// input q = r - v: q_x = r_x (v_x = 0) into u_x, q_y = r_y - v_s into z_y.
__global__ void __launch_bounds__(SCS_BLOCK) scs_update_kernel(const double *__restrict__ zx, double *zy,
                                                               const double *__restrict__ mhx,
                                                               const double *__restrict__ mhy, double *ux,
                                                               const double *__restrict__ uy,
                                                               const double *__restrict__ vy,
                                                               const double *__restrict__ sc, int64_t nx, int64_t ny,
                                                               double alpha, ScsZ z) {
    if (!zrunning(z)) return;
    zx = zmove(zx, z.slot); mhx = zmove(mhx, z.slot); mhy = zmove(mhy, z.slot); ux = zmove(ux, z.slot);
    vy = zmove(vy, z.slot); sc = zmove(sc, z.slot);
    zy = zmove(zy, z.blk); uy = zmove(uy, z.blk);
    const int64_t t = (int64_t)blockIdx.x * SCS_BLOCK + threadIdx.x;
    const double utt = sc[SC_UTT];
    if (t < nx) {
        ux[t] = alpha * (zx[t] - utt * mhx[t]) + (1.0 - alpha) * ux[t];
    } else if (t < nx + ny) {
        const int64_t j = t - nx;
        zy[j] = alpha * (zy[j] - utt * mhy[j]) + (1.0 - alpha) * uy[j] - vy[j];
    }
}

// Cone step after the projection u_y = Pi(q_y): v_s = u_y - q_y; tau and
// kappa from q_tau.
__global__ void __launch_bounds__(SCS_BLOCK) scs_dual_kernel(double *vy, const double *__restrict__ qy,
                                                             const double *__restrict__ uy, double *sc, int64_t ny,
                                                             ScsZ z) {
    if (!zrunning(z)) return;
    vy = zmove(vy, z.slot); sc = zmove(sc, z.slot);
    qy = zmove(qy, z.blk); uy = zmove(uy, z.blk);
    const int64_t t = (int64_t)blockIdx.x * SCS_BLOCK + threadIdx.x;
    if (t < ny) vy[t] = uy[t] - qy[t];
    if (t == 0) {
        const double qt = sc[SC_QT];
        const double ut = fmax(qt, 0.0);
        sc[SC_UT] = ut;
        sc[SC_VK] = ut - qt;
    }
}

// ---- Anderson acceleration of q -> G(q) -----------------------------------
constexpr int AA_MAX = 16;
constexpr int AA_VALS = 3 + 3 * AA_MAX;   // ||f||^2, ||s_j||^2, ||y_j||^2, then per column i:
                                          // s_i^T y_j, s_j^T y_i, s_i^T f

// q as one vector of nq = nx + ny + 1 entries: u_x, z_y, q_tau.
struct QView {
    double *ux, *qy, *sc;
    int64_t nx, ny;
    __device__ __forceinline__ double get(int64_t t) const {
        return t < nx ? ux[t] : (t < nx + ny ? qy[t - nx] : sc[SC_QT]);
    }
    __device__ __forceinline__ void set(int64_t t, double v) const {
        if (t < nx) ux[t] = v;
        else if (t < nx + ny) qy[t - nx] = v;
        else sc[SC_QT] = v;
    }
};

struct AaCols {
    int slot[AA_MAX];
    int count;      // active columns (the new one included)
    int jnew;       // slot of the new pair, -1 if none
};

// f = q_k - G(q_k) (G(q_k) now in q); with a previous input the new pair
// s = q_k - q_prev, y = f - f_prev goes to column jnew; then q_prev = q_k,
// f_prev = f.
__global__ void __launch_bounds__(SCS_BLOCK) aa_pair_kernel(QView q, const double *__restrict__ qk, double *qprev,
                                                            double *fprev, double *S, double *Y, int64_t ld,
                                                            int jnew, int64_t nq) {
    const int64_t t = (int64_t)blockIdx.x * SCS_BLOCK + threadIdx.x;
    if (t >= nq) return;
    const double a = qk[t];
    const double f = a - q.get(t);
    if (jnew >= 0) {
        S[jnew * ld + t] = a - qprev[t];
        Y[jnew * ld + t] = f - fprev[t];
    }
    qprev[t] = a;
    fprev[t] = f;
}

// Block partials of the AA_VALS inner products (unused ones stay 0).
__global__ void __launch_bounds__(SCS_BLOCK) aa_dot_kernel(const double *__restrict__ S, const double *__restrict__ Y,
                                                           int64_t ld, const double *__restrict__ f, AaCols cols,
                                                           int64_t nq, double *part, int parts_ld) {
    double v[AA_VALS];
#pragma unroll
    for (int k = 0; k < AA_VALS; ++k) v[k] = 0.0;
    const int j = cols.jnew;
    for (int64_t t = (int64_t)blockIdx.x * SCS_BLOCK + threadIdx.x; t < nq; t += (int64_t)gridDim.x * SCS_BLOCK) {
        const double ft = f[t];
        v[0] += ft * ft;
        const double sj = j >= 0 ? S[j * ld + t] : 0.0, yj = j >= 0 ? Y[j * ld + t] : 0.0;
        v[1] += sj * sj;
        v[2] += yj * yj;
#pragma unroll
        for (int c = 0; c < AA_MAX; ++c) {
            if (c < cols.count) {
                const int i = cols.slot[c];
                const double si = S[i * ld + t], yi = Y[i * ld + t];
                v[3 + 3 * c] += si * yj;
                v[4 + 3 * c] += sj * yi;
                v[5 + 3 * c] += si * ft;
            }
        }
    }
    __shared__ double red[SCS_BLOCK / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = 0; k < AA_VALS; ++k) {
        double x = v[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        __syncthreads();
        if (lane == 0) red[w] = x;
        __syncthreads();
        if (threadIdx.x == 0) {
            double y = red[0];
            for (int q2 = 1; q2 < SCS_BLOCK / 64; ++q2) y += red[q2];
            part[k * parts_ld + blockIdx.x] = y;
        }
    }
}

// One block of one wave per inner product: out[k] = sum of its partials.
__global__ void __launch_bounds__(64) aa_dot_final_kernel(const double *part, int parts, int parts_ld, double *out) {
    const int k = blockIdx.x, lane = threadIdx.x;
    double x = 0.0;
    for (int q2 = lane; q2 < parts; q2 += 64) x += part[k * parts_ld + q2];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) out[k] = x;
}

struct AaGamma {
    double g[AA_MAX];
    int slot[AA_MAX];
    int count;
};

// Accelerated input q = G(q_k) - (S - Y) gamma; keeps G(q_k) for the
// safeguard and the new input in qk.
__global__ void __launch_bounds__(SCS_BLOCK) aa_extrapolate_kernel(QView q, const double *__restrict__ S,
                                                                   const double *__restrict__ Y, int64_t ld,
                                                                   AaGamma gm, double *qk, double *gsave,
                                                                   int64_t nq) {
    const int64_t t = (int64_t)blockIdx.x * SCS_BLOCK + threadIdx.x;
    if (t >= nq) return;
    const double g = q.get(t);
    double acc = g;
#pragma unroll
    for (int c = 0; c < AA_MAX; ++c)
        if (c < gm.count) {
            const int i = gm.slot[c];
            acc -= gm.g[c] * (S[i * ld + t] - Y[i * ld + t]);
        }
    gsave[t] = g;
    qk[t] = acc;
    q.set(t, acc);
}

// qk = q (a plain step), or q = qk = gsave (a rejected accelerated input).
__global__ void __launch_bounds__(SCS_BLOCK) aa_copy_kernel(QView q, double *qk, const double *gsave, int64_t nq) {
    const int64_t t = (int64_t)blockIdx.x * SCS_BLOCK + threadIdx.x;
    if (t >= nq) return;
    if (gsave) {
        const double g = gsave[t];
        q.set(t, g);
        qk[t] = g;
    } else {
        qk[t] = q.get(t);
    }
}

// Residual partials: rows of the svec (entry 0 of row i is the diagonal),
// then the x range.
__global__ void __launch_bounds__(SCS_BLOCK) scs_resid_kernel(const double *__restrict__ ty,
                                                              const double *__restrict__ vy,
                                                              const double *__restrict__ uy,
                                                              const double *__restrict__ tx,
                                                              const double *__restrict__ ux,
                                                              const double *__restrict__ c,
                                                              const double *__restrict__ sc, int n, int64_t nx,
                                                              double gamma, double *part, ScsZ z) {
    if (!zrunning(z)) return;
    ty = zmove(ty, z.slot); vy = zmove(vy, z.slot); tx = zmove(tx, z.slot); ux = zmove(ux, z.slot);
    c = zmove(c, z.slot); sc = zmove(sc, z.slot); part = zmove(part, z.slot);
    uy = zmove(uy, z.blk);
    const double tau = sc[SC_UT], sigma = sc[SC_SIGMA];
    double m_pri = 0.0, m_ax = 0.0, m_s = 0.0, m_dual = 0.0, m_aty = 0.0, s_cx = 0.0, s_try = 0.0;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int64_t o = svec_col_start(n, i);
        const int len = 2 * (n - i) - 1;
        for (int k = threadIdx.x; k < len; k += SCS_BLOCK) {
            const double a = ty[o + k], s = vy[o + k];
            const double p = a + s - (k == 0 ? tau * gamma : 0.0);
            m_pri = nan_max(m_pri, fabs(p));
            m_ax = nan_max(m_ax, fabs(a));
            m_s = nan_max(m_s, fabs(s));
            if (k == 0) s_try += uy[o];
        }
    }
    for (int64_t t = (int64_t)blockIdx.x * SCS_BLOCK + threadIdx.x; t < nx; t += (int64_t)gridDim.x * SCS_BLOCK) {
        const double a = tx[t];
        m_dual = nan_max(m_dual, fabs(a + sigma * tau * c[t]));
        m_aty = nan_max(m_aty, fabs(a));
        s_cx += c[t] * ux[t];
    }
    double v[R_SLOTS] = {m_pri, m_ax, m_s, m_dual, m_aty, s_cx, s_try};
    const bool mx[R_SLOTS] = {true, true, true, true, true, false, false};
    const int sl[R_SLOTS] = {R_PRI, R_AX, R_S, R_DUAL, R_ATY, R_CX, R_TRY};
    block_reduce<R_SLOTS>(v, mx, sl, part);
}

// Final level: out[k] = reduction of slot k, out[R_SLOTS..] = tau, kappa.
__global__ void __launch_bounds__(64 * R_SLOTS) scs_resid_final_kernel(const double *part, int parts,
                                                                       const double *sc, double *out, ScsZ z) {
    if (!zrunning(z)) return;
    part = zmove(part, z.slot); sc = zmove(sc, z.slot);
    out += 16 * (int64_t)blockIdx.z;
    const int w = threadIdx.x >> 6;
    const double x = sum_parts(part, w, parts, w < R_CX);
    if ((threadIdx.x & 63) == 0) out[w] = x;
    if (threadIdx.x == 0) {
        out[R_SLOTS] = sc[SC_UT];
        out[R_SLOTS + 1] = sc[SC_VK];
    }
}

// Setup reductions over c and G: sum c^2, max |c|, sum diag G.
__global__ void __launch_bounds__(SCS_BLOCK) scs_setup_kernel(const double *__restrict__ c,
                                                              const double *__restrict__ g, int64_t nx, int n,
                                                              double *part) {
    double s2 = 0.0, mc = 0.0, tg = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * SCS_BLOCK + threadIdx.x; t < nx + n; t += (int64_t)gridDim.x * SCS_BLOCK) {
        if (t < nx) {
            s2 += c[t] * c[t];
            mc = nan_max(mc, fabs(c[t]));
        } else {
            tg += g[svec_col_start(n, (int)(t - nx))];
        }
    }
    double v[3] = {s2, mc, tg};
    const bool mx[3] = {false, true, false};
    const int sl[3] = {0, 1, 2};
    block_reduce<3>(v, mx, sl, part);
}

__global__ void __launch_bounds__(64 * 3) scs_final3_kernel(const double *part, int parts, double *out) {
    const int w = threadIdx.x >> 6;
    const double x = sum_parts(part, w, parts, w == 1);
    if ((threadIdx.x & 63) == 0) out[w] = x;
}

// h = (sigma c, gamma 1): hx = sigma c, hy = 0 (the diagonal gamma is added
// by scs_diag_add_kernel in a later launch).
__global__ void __launch_bounds__(SCS_BLOCK) scs_h_kernel(const double *__restrict__ c, double *hx, double *hy,
                                                          int64_t nx, int n, double sigma, double gamma) {
    const int64_t t = (int64_t)blockIdx.x * SCS_BLOCK + threadIdx.x;
    const int64_t ny = (int64_t)n * n;
    if (t < nx) hx[t] = sigma * c[t];
    else if (t < nx + ny) hy[t - nx] = 0.0;
}

// Start: cold u = v = (0, 0, 1); warm u = (x, sigma y, 1), v = (0, s, 0).
__global__ void __launch_bounds__(SCS_BLOCK) scs_start_kernel(const double *x, const double *y, const double *s,
                                                              double *ux, double *uy, double *vy, double *sc,
                                                              int64_t nx, int64_t ny, double sigma, int warm) {
    const int64_t t = (int64_t)blockIdx.x * SCS_BLOCK + threadIdx.x;
    if (t < nx) {
        ux[t] = warm ? x[t] : 0.0;
    } else if (t < nx + ny) {
        const int64_t j = t - nx;
        uy[j] = warm ? sigma * y[j] : 0.0;
        vy[j] = warm ? s[j] : 0.0;
    }
    if (t == 0) {
        sc[SC_UT] = 1.0;
        sc[SC_VK] = warm ? 0.0 : 1.0;
        sc[SC_UTT] = 0.0;
    }
}

// Unscaled outputs x = u_x / tau, y = u_y / (sigma tau), s = v_s / tau; with
// tau = 0 the raw certificate (u_x, u_y, v_s).
__global__ void __launch_bounds__(SCS_BLOCK) scs_out_kernel(const double *__restrict__ ux,
                                                            const double *__restrict__ uy,
                                                            const double *__restrict__ vy, double *x, double *y,
                                                            double *s, const double *__restrict__ sc, int64_t nx,
                                                            int64_t ny, double sigma) {
    const int64_t t = (int64_t)blockIdx.x * SCS_BLOCK + threadIdx.x;
    const double tau = sc[SC_UT];
    const double it = tau > 0.0 ? 1.0 / tau : 1.0, ity = tau > 0.0 ? 1.0 / (sigma * tau) : 1.0;
    if (t < nx) {
        x[t] = ux[t] * it;
    } else if (t < nx + ny) {
        const int64_t j = t - nx;
        y[j] = uy[j] * ity;
        s[j] = vy[j] * it;
    }
}

// W = b - A x with x = u_x / tau (ty = A u_x): w = -ty / tau, then the
// diagonal gamma; post-processing W' = (1 - lam) W + lam gamma 1 scales and
// adds lam gamma to the diagonal.
__global__ void __launch_bounds__(SCS_BLOCK) scs_scale_kernel(const double *in, double *out,
                                                              const double *__restrict__ sc, int64_t ny,
                                                              double factor, int by_tau) {
    const int64_t t = (int64_t)blockIdx.x * SCS_BLOCK + threadIdx.x;
    if (t >= ny) return;
    out[t] = in[t] * (by_tau ? factor / sc[SC_UT] : factor);
}
__global__ void __launch_bounds__(SCS_BLOCK) scs_diag_add_kernel(double *y, int n, double v) {
    const int t = blockIdx.x * SCS_BLOCK + threadIdx.x;
    if (t < n) y[svec_col_start(n, t)] += v;
}

// Sticky status of the cone projections: first non-OK record (instance
// blockIdx.z: record and flag z).
__global__ void scs_fold_kernel(const psd_info *info, int *sticky, ScsZ z) {
    if (!zrunning(z)) return;
    info += blockIdx.z;
    sticky += blockIdx.z;
    if (threadIdx.x == 0 && *sticky == 0 && info->status != 0) *sticky = info->status;
}

// sc[idx] = v (one instance); a[i] = v (the running flags).
__global__ void scs_set_kernel(double *sc, int idx, double v) {
    if (threadIdx.x == 0) sc[idx] = v;
}
__global__ void scs_flag_kernel(int *a, int i, int v) {
    if (threadIdx.x == 0) a[i] = v;
}
__global__ void scs_flags_kernel(int *a, int nb, int v) {
    for (int i = threadIdx.x; i < nb; i += blockDim.x) a[i] = v;
}

// Workspace of a batch of B instances: the projection workspace and the
// Anderson partials are shared (every step runs in stream order); the
// cone-step blocks of the instances are back to back (u_y and z_y, so that
// one batched projection covers them) as are their info records, residual
// and Anderson read-backs and running flags; the rest of an instance's
// vectors, its reduction partials and its affine workspace sit in a slot of
// its own, `inst` bytes apart, so that one launch of each step covers the
// batch (instance = grid z).
struct ScsLayout {
    int d, n, B;
    int64_t nx, ny, nq;
    size_t aff_bytes;
    size_t proj, proj_bytes;
    size_t aapart;
    size_t UY, ZY, PINFO, RED, AAOUT, STICKY, ACTIVE;   // batched, instance b at b * (its size)
    size_t WSAVED;                                        // warm cone steps: the eigen-pair
    size_t slot0, inst;                                   // instance slots
    // offsets inside a slot (the affine workspace and the reduction partials too)
    size_t ux, cv, mhx, zx, tx, vy, mhy, ty, sc, part, aff;
    int m;                                        // Anderson memory (0: off)
    int64_t ld;                                   // stride of the Anderson vectors (doubles)
    size_t qk, qprev, fprev, gsave, S, Y;
    size_t total;
};

bool scs_layout(const psd_scs_settings &s, int B, ScsLayout &L) {
    int64_t nx = 0, ny = 0;
    if (B < 1 || psd_affine_dims(s.d, &nx, &ny) != PSD_OK) return false;
    L.d = s.d;
    L.n = s.d * s.d * s.d * s.d;
    L.B = B;
    L.nx = nx;
    L.ny = ny;
    L.nq = nx + ny + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    if (psd_affine_workspace_size(s.d, &L.aff_bytes) != PSD_OK) return false;
    size_t pb = 0, pg = 0, pm = 0;
    const int32_t n = L.n;
    std::vector<int32_t> sizes(B, n);
    if (psd_workspace_size(1, &n, PSD_FP64_EIG, PSD_FLAG_SAVE, &pb) != PSD_OK) return false;
    if (psd_workspace_size(B, sizes.data(), PSD_FP64_EIG, 0, &pg) != PSD_OK) return false;
    if (s.mixed_iters > 0 && psd_workspace_size(B, sizes.data(), (psd_mode)s.mixed_mode, 0, &pm) != PSD_OK)
        return false;
    L.proj_bytes = std::max(pb, std::max(pg, pm));
    if (s.warm_proj) {
        // warm cone steps: one instance only (the pair is that instance's)
        size_t pw = 0;
        if (B != 1 || psd_workspace_size(1, &n, PSD_FP64_EIG, PSD_FLAG_WARM, &pw) != PSD_OK) return false;
        L.proj_bytes = std::max(L.proj_bytes, pw);
    }
    L.proj = take(L.proj_bytes);
    L.WSAVED = s.warm_proj ? take(psd_saved_size(n)) : 0;
    L.aapart = take(sizeof(double) * SCS_PARTS * AA_VALS);
    const size_t by = sizeof(double) * (size_t)ny, bx = sizeof(double) * (size_t)nx;
    L.UY = take(by * B);
    L.ZY = take(by * B);
    L.PINFO = take(sizeof(psd_info) * B);
    L.RED = take(sizeof(double) * 16 * B);
    L.AAOUT = take(sizeof(double) * AA_VALS * B);
    L.STICKY = take(sizeof(int) * B);
    L.ACTIVE = take(sizeof(int) * B);
    // one instance slot
    size_t o = 0;
    auto slot = [&](size_t bytes) {
        const size_t r = o;
        o += align256(bytes);
        return r;
    };
    L.ux = slot(bx); L.cv = slot(bx); L.mhx = slot(bx); L.zx = slot(bx); L.tx = slot(bx);
    L.vy = slot(by); L.mhy = slot(by); L.ty = slot(by);
    L.sc = slot(sizeof(double) * SC_COUNT);
    L.part = slot(sizeof(double) * SCS_PARTS * R_SLOTS);
    L.aff = slot(L.aff_bytes);
    L.m = s.anderson;
    L.ld = (int64_t)(align256(sizeof(double) * (size_t)L.nq) / sizeof(double));
    L.qk = L.qprev = L.fprev = L.gsave = L.S = L.Y = 0;
    if (L.m > 0) {
        const size_t bq = sizeof(double) * (size_t)L.ld;
        L.qk = slot(bq); L.qprev = slot(bq); L.fprev = slot(bq); L.gsave = slot(bq);
        L.S = slot(bq * L.m);
        L.Y = slot(bq * L.m);
    }
    L.inst = o;
    L.slot0 = off;
    off += L.inst * (size_t)B;
    L.total = off;
    return true;
}

bool settings_ok(const psd_scs_settings *s) {
    return s && s->d >= 2 && s->d <= 8 && s->max_iters >= 1 && s->check_every >= 1 && s->mixed_iters >= 0 &&
           (s->mixed_iters == 0 || s->mixed_mode == PSD_MIXED_BF16 || s->mixed_mode == PSD_MIXED_FP32 ||
            s->mixed_mode == PSD_MIXED_BF16X3) &&
           (s->normalize == 0 || s->normalize == 1) && (s->warm_start == 0 || s->warm_start == 1) &&
           s->anderson >= 0 && s->anderson <= AA_MAX && s->eps >= 0.0 && std::isfinite(s->eps) && s->alpha > 0.0 &&
           s->alpha < 2.0 && s->mixed_switch >= 0.0 && std::isfinite(s->mixed_switch) &&
           (s->warm_proj == 0 || s->warm_proj == 1);
}

int grid_of(int64_t n) { return (int)((n + SCS_BLOCK - 1) / SCS_BLOCK); }

// Solves a x = b (c x c, row-major) by Gaussian elimination with partial
// pivoting; false for a zero pivot or a non-finite result.
bool small_solve(int c, double *a, double *b) {
    for (int k = 0; k < c; ++k) {
        int p = k;
        for (int i = k + 1; i < c; ++i)
            if (std::fabs(a[i * c + k]) > std::fabs(a[p * c + k])) p = i;
        if (!(std::fabs(a[p * c + k]) > 0.0)) return false;
        if (p != k) {
            for (int j = 0; j < c; ++j) std::swap(a[k * c + j], a[p * c + j]);
            std::swap(b[k], b[p]);
        }
        for (int i = k + 1; i < c; ++i) {
            const double l = a[i * c + k] / a[k * c + k];
            for (int j = k; j < c; ++j) a[i * c + j] -= l * a[k * c + j];
            b[i] -= l * b[k];
        }
    }
    for (int k = c - 1; k >= 0; --k) {
        double v = b[k];
        for (int j = k + 1; j < c; ++j) v -= a[k * c + j] * b[j];
        b[k] = v / a[k * c + k];
        if (!std::isfinite(b[k])) return false;
    }
    return true;
}

// Host side of the acceleration: the ring of column slots (oldest first)
// and the inner products S^T Y of the stored pairs.
struct AaHost {
    int m = 0;
    int order[AA_MAX];
    int count = 0;
    bool have_prev = false;
    bool pending = false;     // the input just projected was accelerated
    double nf_save = 0.0;
    double M[AA_MAX][AA_MAX];
    double ss[AA_MAX], yy[AA_MAX];
    int accepted = 0, rejected = 0;
    void reset() {
        count = 0;
        have_prev = false;
        pending = false;
    }
};

// Host view of one instance of a batch.
struct ScsInst {
    double *ux, *cv, *mhx, *zx, *tx, *uy, *vy, *zy, *mhy, *ty, *sc, *red, *aaout, *part;
    void *aff;
    psd_info *pinfo;
    int *sticky;
    double *qk, *qprev, *fprev, *gsave, *S, *Y;
    const double *g;
    double *x, *y, *s, *w;
    double sigma = 1.0, eta = 0.0, b0 = 0.0, c_inf = 0.0;
    psd_scs_info *info;
    AaHost aa;
    int status = PSD_ENOCONV;
    bool done = false;     // converged, failed or stopped: its state is frozen
    bool within = false;   // last check within mixed_switch times the tolerance
};

psd_status scs_solve_batch(const psd_scs_settings *s, int B, const double *g, double *x, double *y, double *sl,
                           double *w, void *ws, size_t ws_bytes, void *stream, psd_scs_info *infos) {
    if (!settings_ok(s) || B < 1 || B > PSD_SCS_MAX_BATCH || !g || !x || !y || !sl || !infos) return PSD_EINVAL;
    ScsLayout L;
    if (!scs_layout(*s, B, L)) return PSD_EINVAL;
    if (!ws || ws_bytes < L.total) return PSD_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % 256) return PSD_EINVAL;
    for (const void *p : {(const void *)g, (const void *)x, (const void *)y, (const void *)sl, (const void *)w})
        if (p && (reinterpret_cast<uintptr_t>(p) & 7u)) return PSD_EINVAL;
    {   // g, x, y, s, w (each B vectors back to back) pairwise disjoint
        const size_t bx = sizeof(double) * (size_t)L.nx * B, by = sizeof(double) * (size_t)L.ny * B;
        const char *pp[5] = {(const char *)g, (const char *)x, (const char *)y, (const char *)sl, (const char *)w};
        const size_t nb[5] = {by, bx, by, by, by};
        for (int i = 0; i < 5; ++i)
            for (int j = i + 1; j < 5; ++j)
                if (pp[i] && pp[j] && pp[i] < pp[j] + nb[j] && pp[j] < pp[i] + nb[i]) return PSD_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);
    auto D = [&](size_t off) { return reinterpret_cast<double *>(base + off); };
    void *proj = base + L.proj;
    double *aapart = D(L.aapart);
    double *UY = D(L.UY), *ZY = D(L.ZY), *RED = D(L.RED), *AAOUT = D(L.AAOUT);
    psd_info *PINFO = reinterpret_cast<psd_info *>(base + L.PINFO);
    int *STICKY = reinterpret_cast<int *>(base + L.STICKY);
    int *ACTIVE = reinterpret_cast<int *>(base + L.ACTIVE);
    double *WSAVED = s->warm_proj ? D(L.WSAVED) : nullptr;
    bool have_pair = false;   // WSAVED holds the pair of the previous FP64 cone step
    int warm_wait = 0, warm_backoff = 0, warm_refined = 0, warm_fallbacks = 0;
    const int d = L.d, n = L.n;
    const int64_t nx = L.nx, ny = L.ny, nq = L.nq;
    const double gamma = 1.0 / (double)(d * d);
    const double alpha = s->alpha;
    std::vector<ScsInst> inst(B);
    for (int b = 0; b < B; ++b) {
        ScsInst &I = inst[b];
        char *sb = base + L.slot0 + L.inst * (size_t)b;
        auto S_ = [&](size_t off) { return reinterpret_cast<double *>(sb + off); };
        I.ux = S_(L.ux); I.cv = S_(L.cv); I.mhx = S_(L.mhx); I.zx = S_(L.zx); I.tx = S_(L.tx);
        I.vy = S_(L.vy); I.mhy = S_(L.mhy); I.ty = S_(L.ty); I.sc = S_(L.sc);
        I.part = S_(L.part);
        I.aff = sb + L.aff;
        I.uy = UY + ny * b;
        I.zy = ZY + ny * b;
        I.red = RED + 16 * b;
        I.aaout = AAOUT + AA_VALS * b;
        I.pinfo = PINFO + b;
        I.sticky = STICKY + b;
        I.qk = L.m ? S_(L.qk) : nullptr; I.qprev = L.m ? S_(L.qprev) : nullptr;
        I.fprev = L.m ? S_(L.fprev) : nullptr; I.gsave = L.m ? S_(L.gsave) : nullptr;
        I.S = L.m ? S_(L.S) : nullptr; I.Y = L.m ? S_(L.Y) : nullptr;
        I.g = g + ny * b;
        I.x = x + nx * b;
        I.y = y + ny * b;
        I.s = sl + ny * b;
        I.w = w ? w + ny * b : nullptr;
        I.info = infos + b;
        *I.info = psd_scs_info{};
        I.aa.m = L.m;
    }

#define SCS_TRY(call)                                    \
    do {                                                 \
        const psd_status e_ = (call);                    \
        if (e_ != PSD_OK) return e_;                     \
    } while (0)
#define SCS_LAUNCHED()                                   \
    do {                                                 \
        if (hipGetLastError() != hipSuccess) return PSD_EDEVICE; \
    } while (0)
#define SCS_READ(dst, src, bytes)                                                          \
    do {                                                                                   \
        if (hipMemcpyAsync((dst), (src), (bytes), hipMemcpyDeviceToHost, st) != hipSuccess || \
            hipStreamSynchronize(st) != hipSuccess)                                        \
            return PSD_EDEVICE;                                                            \
    } while (0)

    // ---- setup: c = A^T G, norms, sigma, M^-1 h, eta (per instance) ---------
    const int parts_x = std::min<int64_t>(SCS_PARTS, std::max<int64_t>(1, grid_of(nx + n)));
    const ScsZ one{0, 0, nullptr};
    for (int b = 0; b < B; ++b) {
        ScsInst &I = inst[b];
        SCS_TRY(psd_constraint_adjoint(d, I.g, I.cv, I.aff, L.aff_bytes, st));
        hipLaunchKernelGGL(scs_setup_kernel, dim3(parts_x), dim3(SCS_BLOCK), 0, st, I.cv, I.g, nx, n, I.part);
        hipLaunchKernelGGL(scs_final3_kernel, dim3(1), dim3(64 * 3), 0, st, I.part, parts_x, I.red);
    }
    SCS_LAUNCHED();
    std::vector<double> host(16 * (size_t)B);
    SCS_READ(host.data(), RED, sizeof(double) * 16 * B);
    for (int b = 0; b < B; ++b) {
        ScsInst &I = inst[b];
        const double *h3 = &host[16 * b];
        const double c_norm = std::sqrt(h3[0]);
        I.c_inf = h3[1];
        I.b0 = gamma * h3[2];
        const double b_norm = gamma * std::sqrt((double)n);
        I.sigma = (s->normalize && c_norm > 0.0) ? b_norm / c_norm : 1.0;
        I.info->sigma = I.sigma;
        if (!std::isfinite(c_norm) || !std::isfinite(I.b0)) {
            I.status = PSD_ENONFINITE;
            I.done = true;
            continue;
        }
        hipLaunchKernelGGL(scs_h_kernel, dim3(grid_of(nx + ny)), dim3(SCS_BLOCK), 0, st, I.cv, I.mhx, I.mhy, nx, n,
                           I.sigma, gamma);
        hipLaunchKernelGGL(scs_diag_add_kernel, dim3(grid_of(n)), dim3(SCS_BLOCK), 0, st, I.mhy, n, gamma);
        hipLaunchKernelGGL(scs_set_kernel, dim3(1), dim3(64), 0, st, I.sc, (int)SC_SIGMA, I.sigma);
        SCS_LAUNCHED();
        SCS_TRY(psd_affine_step(d, I.mhx, I.mhy, I.mhx, I.mhy, I.aff, L.aff_bytes, st));
        hipLaunchKernelGGL(scs_dot_kernel, dim3(parts_x), dim3(SCS_BLOCK), 0, st, I.cv, I.mhx, I.mhy, nx, n,
                           (const double *)I.sc, gamma, I.part, one);
        hipLaunchKernelGGL(scs_final3_kernel, dim3(1), dim3(64 * 3), 0, st, I.part, parts_x, I.red);
    }
    SCS_LAUNCHED();
    SCS_READ(host.data(), RED, sizeof(double) * 16 * B);
    for (int b = 0; b < B; ++b) {
        ScsInst &I = inst[b];
        if (I.done) continue;
        I.eta = host[16 * b];
        if (!std::isfinite(I.eta)) {
            I.status = PSD_ENONFINITE;
            I.done = true;
            continue;
        }
        hipLaunchKernelGGL(scs_start_kernel, dim3(grid_of(nx + ny)), dim3(SCS_BLOCK), 0, st, I.x, I.y, I.s, I.ux,
                           I.uy, I.vy, I.sc, nx, ny, I.sigma, s->warm_start);
        hipLaunchKernelGGL(scs_set_kernel, dim3(1), dim3(64), 0, st, I.sc, (int)SC_ETA, I.eta);
    }
    hipLaunchKernelGGL(scs_flags_kernel, dim3(1), dim3(256), 0, st, ACTIVE, B, 1);
    for (int b = 0; b < B; ++b)
        if (inst[b].done) hipLaunchKernelGGL(scs_flag_kernel, dim3(1), dim3(64), 0, st, ACTIVE, b, 0);
    if (hipMemsetAsync(STICKY, 0, sizeof(int) * B, st) != hipSuccess) return PSD_EDEVICE;
    for (int b = 0; b < B; ++b)   // an instance stopped at setup still has a block in the batched projection
        if (inst[b].done && hipMemsetAsync(inst[b].zy, 0, sizeof(double) * (size_t)ny, st) != hipSuccess)
            return PSD_EDEVICE;
    SCS_LAUNCHED();

    // One launch per step for the whole batch (instance = grid z); the
    // instances that stopped are skipped by their flags.
    ScsInst &I0 = inst[0];
    const ScsZ zb{(int64_t)L.inst, (int64_t)(sizeof(double) * ny), ACTIVE};
    const int64_t xs = (int64_t)(L.inst / sizeof(double));
    // the cone input q = u~_r - v of the current (u, v): (u_x, z_y, q_tau)
    auto cone_input = [&]() -> psd_status {
        hipLaunchKernelGGL(scs_sum_kernel, dim3(grid_of(nx + ny), 1, B), dim3(SCS_BLOCK), 0, st, I0.ux, UY, I0.vy,
                           I0.zx, ZY, nx, ny, zb);
        if (hipGetLastError() != hipSuccess) return PSD_EDEVICE;
        if (affine_step_batched(d, I0.zx, ZY, I0.zx, ZY, xs, ny, I0.aff, (int64_t)L.inst, B, ACTIVE, st) != hipSuccess)
            return PSD_EDEVICE;
        hipLaunchKernelGGL(scs_dot_kernel, dim3(parts_x, 1, B), dim3(SCS_BLOCK), 0, st, I0.cv, I0.zx, ZY, nx, n,
                           (const double *)I0.sc, gamma, I0.part, zb);
        hipLaunchKernelGGL(scs_tau_kernel, dim3(1, 1, B), dim3(64), 0, st, I0.part, parts_x, I0.sc, alpha, zb);
        hipLaunchKernelGGL(scs_update_kernel, dim3(grid_of(nx + ny), 1, B), dim3(SCS_BLOCK), 0, st, I0.zx, ZY, I0.mhx,
                           I0.mhy, I0.ux, UY, I0.vy, I0.sc, nx, ny, alpha, zb);
        return hipGetLastError() == hipSuccess ? PSD_OK : PSD_EDEVICE;
    };

    // Anderson, first half: the new pair and the inner products (device)
    const int aa_parts = std::min<int64_t>(SCS_PARTS, std::max<int64_t>(1, grid_of(nq)));
    std::vector<AaCols> cols(B);
    std::vector<int> jnew(B, -1), evict(B, -1);
    auto anderson_launch = [&](int b) -> psd_status {
        ScsInst &I = inst[b];
        const QView qv{I.ux, I.zy, I.sc, nx, ny};
        jnew[b] = evict[b] = -1;
        if (I.aa.have_prev) {
            if (I.aa.count < I.aa.m) {
                bool used[AA_MAX] = {};
                for (int c = 0; c < I.aa.count; ++c) used[I.aa.order[c]] = true;
                for (int i = 0; i < I.aa.m; ++i)
                    if (!used[i]) { jnew[b] = i; break; }
            } else {
                jnew[b] = evict[b] = I.aa.order[0];
            }
        }
        hipLaunchKernelGGL(aa_pair_kernel, dim3(grid_of(nq)), dim3(SCS_BLOCK), 0, st, qv, I.qk, I.qprev, I.fprev,
                           I.S, I.Y, L.ld, jnew[b], nq);
        AaCols &cl = cols[b];
        cl = AaCols{};
        int ncols = 0;
        for (int c = 0; c < I.aa.count; ++c)
            if (I.aa.order[c] != evict[b]) cl.slot[ncols++] = I.aa.order[c];
        if (jnew[b] >= 0) cl.slot[ncols++] = jnew[b];
        cl.count = ncols;
        cl.jnew = jnew[b];
        hipLaunchKernelGGL(aa_dot_kernel, dim3(aa_parts), dim3(SCS_BLOCK), 0, st, I.S, I.Y, L.ld, I.fprev, cl, nq,
                           aapart, SCS_PARTS);
        hipLaunchKernelGGL(aa_dot_final_kernel, dim3(3 + 3 * ncols), dim3(64), 0, st, aapart, aa_parts, SCS_PARTS,
                           I.aaout);
        return hipGetLastError() == hipSuccess ? PSD_OK : PSD_EDEVICE;
    };
    // Anderson, second half: the host decision and the next input
    auto anderson_finish = [&](int b, const double *v) -> psd_status {
        ScsInst &I = inst[b];
        const QView qv{I.ux, I.zy, I.sc, nx, ny};
        const AaCols &cl = cols[b];
        const int ncols = cl.count;
        const double nf = std::sqrt(v[0]);
        if (I.aa.pending) {
            I.aa.pending = false;
            if (!(nf <= 2.0 * I.aa.nf_save)) {      // safeguard: back to the plain input
                hipLaunchKernelGGL(aa_copy_kernel, dim3(grid_of(nq)), dim3(SCS_BLOCK), 0, st, qv, I.qk, I.gsave, nq);
                I.aa.reset();
                ++I.aa.rejected;
                return hipGetLastError() == hipSuccess ? PSD_OK : PSD_EDEVICE;
            }
        }
        if (jnew[b] >= 0) {
            for (int c = 0; c < ncols; ++c) {
                const int i = cl.slot[c];
                I.aa.M[i][jnew[b]] = v[3 + 3 * c];   // s_i^T y_j
                I.aa.M[jnew[b]][i] = v[4 + 3 * c];   // s_j^T y_i
            }
            I.aa.ss[jnew[b]] = v[1];
            I.aa.yy[jnew[b]] = v[2];
            for (int c = 0; c < ncols; ++c) I.aa.order[c] = cl.slot[c];
            I.aa.count = ncols;
        }
        I.aa.have_prev = true;
        bool step = I.aa.count > 0;
        AaGamma gm{};
        if (step) {
            const int c = I.aa.count;
            double A[AA_MAX * AA_MAX], bb[AA_MAX], s2 = 0.0, y2 = 0.0;
            for (int q = 0; q < c; ++q) {
                s2 += I.aa.ss[I.aa.order[q]];
                y2 += I.aa.yy[I.aa.order[q]];
            }
            const double lam = 1e-8 * std::sqrt(s2) * std::sqrt(y2);
            for (int q = 0; q < c; ++q) {
                for (int r2 = 0; r2 < c; ++r2)
                    A[q * c + r2] = I.aa.M[I.aa.order[q]][I.aa.order[r2]] + (q == r2 ? lam : 0.0);
                bb[q] = v[5 + 3 * q];              // s_i^T f, columns in the order above
            }
            step = small_solve(c, A, bb);
            for (int q = 0; step && q < c; ++q) step = std::fabs(bb[q]) <= 1e10;
            if (step) {
                for (int q = 0; q < c; ++q) {
                    gm.g[q] = bb[q];
                    gm.slot[q] = I.aa.order[q];
                }
                gm.count = c;
            }
        }
        if (step) {
            hipLaunchKernelGGL(aa_extrapolate_kernel, dim3(grid_of(nq)), dim3(SCS_BLOCK), 0, st, qv, I.S, I.Y, L.ld,
                               gm, I.qk, I.gsave, nq);
            I.aa.pending = true;
            I.aa.nf_save = nf;
            ++I.aa.accepted;
        } else {
            hipLaunchKernelGGL(aa_copy_kernel, dim3(grid_of(nq)), dim3(SCS_BLOCK), 0, st, qv, I.qk, nullptr, nq);
        }
        return hipGetLastError() == hipSuccess ? PSD_OK : PSD_EDEVICE;
    };

    // the unscaled outputs of an instance, written when it stops (later
    // batched projections may recompute its u_y in another mode)
    auto write_outputs = [&](ScsInst &I) {
        hipLaunchKernelGGL(scs_out_kernel, dim3(grid_of(nx + ny)), dim3(SCS_BLOCK), 0, st, I.ux, I.uy, I.vy, I.x, I.y,
                           I.s, I.sc, nx, ny, I.sigma);
    };

    // ---- iterations -------------------------------------------------------
    const int parts_r = std::min(SCS_PARTS, std::max(n, 1));
    const double bound_b = gamma;   // ||b||_inf
    std::vector<int32_t> sizes(B, n);
    std::vector<double> aa_host((size_t)AA_VALS * B);
    bool switched = false;          // the batch left the mixed cone steps
    int k = 0;
    SCS_TRY(cone_input());
    for (int b = 0; b < B; ++b) {
        if (inst[b].done) continue;
        if (L.m) hipLaunchKernelGGL(aa_copy_kernel, dim3(grid_of(nq)), dim3(SCS_BLOCK), 0, st,
                                    QView{inst[b].ux, inst[b].zy, inst[b].sc, nx, ny}, inst[b].qk, nullptr, nq);
    }
    SCS_LAUNCHED();
    int last = 0;
    for (k = 1; k <= s->max_iters; ++k) {
        // cone step of every instance: u_y = Pi(q_y) in one batched call
        // (cheaper than calls over the runs of running instances, whose
        // smaller groups are latency-bound: a stopped instance's block is
        // projected again, its outputs already written), then v_s = u_y - q_y,
        // tau, kappa for the running ones
        const psd_mode mode = (k <= s->mixed_iters && !switched) ? (psd_mode)s->mixed_mode : PSD_FP64_EIG;
        if (WSAVED && mode == PSD_FP64_EIG) {
            // warm cone steps: from the eigen-pair the previous FP64 step left
            // (psd_project_warm falls back to the cold path by itself).  After
            // a fallback the next 1, 2, 4 .. 16 steps (doubling while attempts
            // keep failing) go cold, the last of them saving its pair: inputs
            // that jump (early iterations, accelerated steps) then cost no
            // refinement attempt each.
            if (have_pair && warm_wait == 0) {
                SCS_TRY(psd_project_warm(n, ZY, UY, WSAVED, WSAVED, proj, L.proj_bytes, st, PINFO));
                psd_info pi{};
                SCS_READ(&pi, PINFO, sizeof pi);
                if (pi.fallback) {
                    ++warm_fallbacks;
                    warm_backoff = std::min(16, std::max(1, 2 * warm_backoff));
                    warm_wait = warm_backoff;
                } else {
                    ++warm_refined;
                    warm_backoff = 0;
                }
            } else {
                const bool save = warm_wait <= 1;
                SCS_TRY(psd_project(n, ZY, UY, PSD_FP64_EIG, proj, L.proj_bytes, st, PINFO, save ? WSAVED : nullptr));
                have_pair = save;
                if (warm_wait > 0) --warm_wait;
            }
        } else {
            SCS_TRY(psd_project_batched(B, sizes.data(), ZY, UY, mode, proj, L.proj_bytes, st, PINFO));
        }
        hipLaunchKernelGGL(scs_fold_kernel, dim3(1, 1, B), dim3(64), 0, st, PINFO, STICKY, zb);
        hipLaunchKernelGGL(scs_dual_kernel, dim3(grid_of(ny), 1, B), dim3(SCS_BLOCK), 0, st, I0.vy, ZY, UY, I0.sc, ny,
                           zb);
        SCS_LAUNCHED();
        last = k;
        if (k % s->check_every == 0 || k == s->max_iters) {
            if (constraint_apply_batched(d, I0.ux, I0.ty, xs, xs, I0.aff, (int64_t)L.inst, B, ACTIVE, st) != hipSuccess ||
                constraint_adjoint_batched(d, UY, I0.tx, ny, xs, I0.aff, (int64_t)L.inst, B, ACTIVE, st) != hipSuccess)
                return PSD_EDEVICE;
            hipLaunchKernelGGL(scs_resid_kernel, dim3(parts_r, 1, B), dim3(SCS_BLOCK), 0, st, I0.ty, I0.vy, UY, I0.tx,
                               I0.ux, I0.cv, I0.sc, n, nx, gamma, I0.part, zb);
            hipLaunchKernelGGL(scs_resid_final_kernel, dim3(1, 1, B), dim3(64 * R_SLOTS), 0, st, I0.part, parts_r,
                               I0.sc, RED, zb);
            SCS_LAUNCHED();
            SCS_READ(host.data(), RED, sizeof(double) * 16 * B);
            bool all_within = true;
            for (int b = 0; b < B; ++b) {
                ScsInst &I = inst[b];
                if (I.done) continue;
                const double *r = &host[16 * b];
                const double tau = r[R_SLOTS], kappa = r[R_SLOTS + 1];
                I.info->tau = tau;
                I.info->kappa = kappa;
                I.info->iters = k;
                bool finite = std::isfinite(tau) && std::isfinite(kappa);
                for (int q2 = 0; q2 < R_SLOTS; ++q2) finite = finite && std::isfinite(r[q2]);
                if (!finite) {
                    I.status = PSD_ENONFINITE;
                    I.done = true;
                    write_outputs(I);
                    hipLaunchKernelGGL(scs_flag_kernel, dim3(1), dim3(64), 0, st, ACTIVE, b, 0);
                    continue;
                }
                I.within = false;
                if (tau > 0.0) {
                    const double it = 1.0 / tau, ist = 1.0 / (I.sigma * tau);
                    const double res_pri = r[R_PRI] * it, ax_inf = r[R_AX] * it, s_inf = r[R_S] * it;
                    const double res_dual = r[R_DUAL] * ist, aty_inf = r[R_ATY] * ist;
                    const double cx = r[R_CX] * it, by = gamma * r[R_TRY] * ist;
                    const double gap = std::fabs(cx + by);
                    I.info->res_pri = res_pri;
                    I.info->res_dual = res_dual;
                    I.info->gap = gap;
                    I.info->pobj = I.b0 - cx;
                    I.info->dobj = I.b0 + by;
                    const double e = s->eps;
                    const double bp = e + e * std::max(ax_inf, std::max(s_inf, bound_b));
                    const double bd = e + e * std::max(aty_inf, I.c_inf);
                    const double bg = e + e * std::max(std::fabs(cx), std::fabs(by));
                    if (e > 0.0 && res_pri <= bp && res_dual <= bd && gap <= bg) {
                        I.status = PSD_OK;
                        I.done = true;
                        write_outputs(I);
                        hipLaunchKernelGGL(scs_flag_kernel, dim3(1), dim3(64), 0, st, ACTIVE, b, 0);
                        continue;
                    }
                    const double ms = s->mixed_switch;
                    I.within = ms > 0.0 && e > 0.0 && res_pri <= ms * bp && res_dual <= ms * bd && gap <= ms * bg;
                } else {
                    I.info->res_pri = I.info->res_dual = I.info->gap = INFINITY;
                }
                all_within = all_within && I.within;
            }
            if (!switched && k <= s->mixed_iters && s->mixed_switch > 0.0 && all_within) {
                bool any = false;
                for (int b = 0; b < B; ++b) any = any || !inst[b].done;
                if (any) {
                    switched = true;
                    for (int b = 0; b < B; ++b)
                        if (!inst[b].done) inst[b].info->switch_iter = k;
                }
            }
        }
        bool any = false;
        for (int b = 0; b < B; ++b) any = any || !inst[b].done;
        if (!any || k == s->max_iters) break;
        SCS_TRY(cone_input());
        if (L.m) {
            for (int b = 0; b < B; ++b)
                if (!inst[b].done) SCS_TRY(anderson_launch(b));
            SCS_READ(aa_host.data(), AAOUT, sizeof(double) * AA_VALS * B);
        }
        if (L.m)
            for (int b = 0; b < B; ++b)
                if (!inst[b].done) SCS_TRY(anderson_finish(b, &aa_host[(size_t)AA_VALS * b]));
    }
    std::vector<int> stick(B, 0);
    SCS_READ(stick.data(), STICKY, sizeof(int) * B);
    for (int b = 0; b < B; ++b) {
        ScsInst &I = inst[b];
        if (I.info->iters == 0) I.info->iters = last;
        I.info->aa_accepted = I.aa.accepted;
        I.info->aa_rejected = I.aa.rejected;
        I.info->proj_status = stick[b];
        if (I.status == PSD_OK && stick[b] == PSD_ENONFINITE) I.status = PSD_ENONFINITE;
        if (!I.done) write_outputs(I);
    }
    SCS_LAUNCHED();

    // ---- post-processing of W = b - A x (App. "Sparse SDP formulation") --
    for (int b = 0; b < B && w; ++b) {
        ScsInst &I = inst[b];
        if (!(I.info->tau > 0.0) || I.status == PSD_ENONFINITE) continue;
        SCS_TRY(psd_constraint_apply(d, I.ux, I.ty, I.aff, L.aff_bytes, st));
        hipLaunchKernelGGL(scs_scale_kernel, dim3(grid_of(ny)), dim3(SCS_BLOCK), 0, st, I.ty, I.w, I.sc, ny, -1.0, 1);
        hipLaunchKernelGGL(scs_diag_add_kernel, dim3(grid_of(n)), dim3(SCS_BLOCK), 0, st, I.w, n, gamma);
        SCS_LAUNCHED();
        // lambda_min(W) from the saved eigenvalues (ascending) of an FP64 projection
        double *saved = static_cast<double *>(I.aff);
        SCS_TRY(psd_project(n, I.w, I.zy, PSD_FP64_EIG, proj, L.proj_bytes, st, I.pinfo, saved));
        double lmin = 0.0;
        psd_info pi{};
        if (hipMemcpyAsync(&lmin, saved, sizeof lmin, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&pi, I.pinfo, sizeof pi, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return PSD_EDEVICE;
        double lam = 0.0;
        if (pi.status == PSD_OK && lmin < 0.0) {
            lam = -lmin / (gamma - lmin);
            hipLaunchKernelGGL(scs_scale_kernel, dim3(grid_of(ny)), dim3(SCS_BLOCK), 0, st, I.w, I.w, I.sc, ny,
                               1.0 - lam, 0);
            hipLaunchKernelGGL(scs_diag_add_kernel, dim3(grid_of(n)), dim3(SCS_BLOCK), 0, st, I.w, n, lam * gamma);
            SCS_LAUNCHED();
        }
        I.info->post_lambda = lam;
        I.info->post_lambda_min = lmin;
    }
    for (int b = 0; b < B; ++b) inst[b].info->status = inst[b].status;
    if (WSAVED) {
        inst[0].info->warm_refined = warm_refined;
        inst[0].info->warm_fallbacks = warm_fallbacks;
    }
#undef SCS_TRY
#undef SCS_LAUNCHED
#undef SCS_READ
    return PSD_OK;
}

}  // namespace

}  // namespace psd

using namespace psd;

extern "C" {

psd_status psd_scs_workspace_size(const psd_scs_settings *s, size_t *bytes) {
    return psd_scs_workspace_size_batched(s, 1, bytes);
}

psd_status psd_scs_workspace_size_batched(const psd_scs_settings *s, int32_t nbatch, size_t *bytes) {
    if (!settings_ok(s) || !bytes || nbatch < 1 || nbatch > PSD_SCS_MAX_BATCH) return PSD_EINVAL;
    ScsLayout L;
    if (!scs_layout(*s, nbatch, L)) return PSD_EINVAL;
    *bytes = L.total;
    return PSD_OK;
}

psd_status psd_scs_solve(const psd_scs_settings *s, const double *g, double *x, double *y, double *s_out, double *w,
                         void *ws, size_t ws_bytes, void *stream, psd_scs_info *info) {
    return scs_solve_batch(s, 1, g, x, y, s_out, w, ws, ws_bytes, stream, info);
}

psd_status psd_scs_solve_batched(const psd_scs_settings *s, int32_t nbatch, const double *g, double *x, double *y,
                                 double *s_out, double *w, void *ws, size_t ws_bytes, void *stream,
                                 psd_scs_info *infos) {
    return scs_solve_batch(s, nbatch, g, x, y, s_out, w, ws, ws_bytes, stream, infos);
}

}  // extern "C"
