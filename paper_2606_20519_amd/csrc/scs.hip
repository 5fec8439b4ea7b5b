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

#include "../../include/psdproj.h"
#include "common.h"

namespace psd {

namespace {

static_assert(sizeof(psd_scs_settings) == 56, "psd_scs_settings layout");
static_assert(sizeof(psd_scs_info) == 104, "psd_scs_info layout");

constexpr int SCS_BLOCK = 256;
constexpr int SCS_PARTS = 512;   // blocks of the first reduction level

// Device scalars of the iteration.
enum { SC_UT = 0, SC_VK = 1, SC_UTT = 2, SC_QT = 3, SC_COUNT = 8 };
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
                                                            int64_t nx, int64_t ny) {
    const int64_t t = (int64_t)blockIdx.x * SCS_BLOCK + threadIdx.x;
    if (t < nx) zx[t] = ux[t];
    else if (t < nx + ny) zy[t - nx] = uy[t - nx] + vy[t - nx];
}

// Partial sums of h^T z = sigma c^T z_x + gamma tr(z_y) into part[0 ..).
__global__ void __launch_bounds__(SCS_BLOCK) scs_dot_kernel(const double *__restrict__ c,
                                                            const double *__restrict__ zx,
                                                            const double *__restrict__ zy, int64_t nx, int n,
                                                            double sigma, double gamma, double *part) {
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
__global__ void __launch_bounds__(64) scs_tau_kernel(const double *part, int parts, double *sc, double eta,
                                                     double alpha) {
    const double hz = sum_parts(part, 0, parts, false);
    if (threadIdx.x != 0) return;
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
                                                               double alpha) {
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
                                                             const double *__restrict__ uy, double *sc, int64_t ny) {
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
                                                              double sigma, double gamma, double *part) {
    const double tau = sc[SC_UT];
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
                                                                       const double *sc, double *out) {
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

// Sticky status of the cone projections: first non-OK record.
__global__ void scs_fold_kernel(const psd_info *info, int *sticky) {
    if (threadIdx.x == 0 && *sticky == 0 && info->status != 0) *sticky = info->status;
}

struct ScsLayout {
    int d, n;
    int64_t nx, ny, nq;
    size_t ux, cv, mhx, zx, tx;           // nx each
    size_t uy, vy, zy, mhy, ty;           // ny each
    size_t aff, aff_bytes;
    size_t proj, proj_bytes;
    size_t part, sc, red, pinfo, sticky;
    int m;                                // Anderson memory (0: off)
    int64_t ld;                           // stride of the Anderson vectors (doubles)
    size_t qk, qprev, fprev, gsave, S, Y, aapart, aaout;
    size_t total;
};

bool scs_layout(const psd_scs_settings &s, ScsLayout &L) {
    int64_t nx = 0, ny = 0;
    if (psd_affine_dims(s.d, &nx, &ny) != PSD_OK) return false;
    L.d = s.d;
    L.n = s.d * s.d * s.d * s.d;
    L.nx = nx;
    L.ny = ny;
    L.nq = nx + ny + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t bx = sizeof(double) * (size_t)nx, by = sizeof(double) * (size_t)ny;
    L.ux = take(bx); L.cv = take(bx); L.mhx = take(bx); L.zx = take(bx); L.tx = take(bx);
    L.uy = take(by); L.vy = take(by); L.zy = take(by); L.mhy = take(by); L.ty = take(by);
    if (psd_affine_workspace_size(s.d, &L.aff_bytes) != PSD_OK) return false;
    L.aff = take(L.aff_bytes);
    size_t pb = 0, pm = 0;
    const int32_t n = L.n;
    if (psd_workspace_size(1, &n, PSD_FP64_EIG, PSD_FLAG_SAVE, &pb) != PSD_OK) return false;
    if (s.mixed_iters > 0 && psd_workspace_size(1, &n, (psd_mode)s.mixed_mode, 0, &pm) != PSD_OK) return false;
    L.proj_bytes = std::max(pb, pm);
    L.proj = take(L.proj_bytes);
    L.part = take(sizeof(double) * SCS_PARTS * R_SLOTS);
    L.sc = take(sizeof(double) * SC_COUNT);
    L.red = take(sizeof(double) * 16);
    L.pinfo = take(sizeof(psd_info));
    L.sticky = take(sizeof(int));
    L.m = s.anderson;
    L.ld = (int64_t)(align256(sizeof(double) * (size_t)L.nq) / sizeof(double));
    L.qk = L.qprev = L.fprev = L.gsave = L.S = L.Y = L.aapart = L.aaout = 0;
    if (L.m > 0) {
        const size_t bq = sizeof(double) * (size_t)L.ld;
        L.qk = take(bq); L.qprev = take(bq); L.fprev = take(bq); L.gsave = take(bq);
        L.S = take(bq * L.m);
        L.Y = take(bq * L.m);
        L.aapart = take(sizeof(double) * SCS_PARTS * AA_VALS);
        L.aaout = take(sizeof(double) * AA_VALS);
    }
    L.total = off;
    return true;
}

bool settings_ok(const psd_scs_settings *s) {
    return s && s->d >= 2 && s->d <= 8 && s->max_iters >= 1 && s->check_every >= 1 && s->mixed_iters >= 0 &&
           (s->mixed_iters == 0 || s->mixed_mode == PSD_MIXED_BF16 || s->mixed_mode == PSD_MIXED_FP32 ||
            s->mixed_mode == PSD_MIXED_BF16X3) &&
           (s->normalize == 0 || s->normalize == 1) && (s->warm_start == 0 || s->warm_start == 1) &&
           s->anderson >= 0 && s->anderson <= AA_MAX && s->eps >= 0.0 && std::isfinite(s->eps) && s->alpha > 0.0 &&
           s->alpha < 2.0 && s->mixed_switch >= 0.0 && std::isfinite(s->mixed_switch);
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

}  // namespace

}  // namespace psd

using namespace psd;

extern "C" {

psd_status psd_scs_workspace_size(const psd_scs_settings *s, size_t *bytes) {
    if (!settings_ok(s) || !bytes) return PSD_EINVAL;
    ScsLayout L;
    if (!scs_layout(*s, L)) return PSD_EINVAL;
    *bytes = L.total;
    return PSD_OK;
}

psd_status psd_scs_solve(const psd_scs_settings *s, const double *g, double *x, double *y, double *sl, double *w,
                         void *ws, size_t ws_bytes, void *stream, psd_scs_info *info) {
    if (!settings_ok(s) || !g || !x || !y || !sl || !info) return PSD_EINVAL;
    ScsLayout L;
    if (!scs_layout(*s, L)) return PSD_EINVAL;
    if (!ws || ws_bytes < L.total) return PSD_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % 256) return PSD_EINVAL;
    for (const void *p : {(const void *)g, (const void *)x, (const void *)y, (const void *)sl, (const void *)w})
        if (p && (reinterpret_cast<uintptr_t>(p) & 7u)) return PSD_EINVAL;
    {   // x, y, s, w, g pairwise disjoint
        const size_t bx = sizeof(double) * (size_t)L.nx, by = sizeof(double) * (size_t)L.ny;
        const char *pp[5] = {(const char *)g, (const char *)x, (const char *)y, (const char *)sl, (const char *)w};
        const size_t nb[5] = {by, bx, by, by, by};
        for (int i = 0; i < 5; ++i)
            for (int j = i + 1; j < 5; ++j)
                if (pp[i] && pp[j] && pp[i] < pp[j] + nb[j] && pp[j] < pp[i] + nb[i]) return PSD_EINVAL;
    }
    *info = psd_scs_info{};
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);
    auto D = [&](size_t off) { return reinterpret_cast<double *>(base + off); };
    double *ux = D(L.ux), *cv = D(L.cv), *mhx = D(L.mhx), *zx = D(L.zx), *tx = D(L.tx);
    double *uy = D(L.uy), *vy = D(L.vy), *zy = D(L.zy), *mhy = D(L.mhy), *ty = D(L.ty);
    void *aff = base + L.aff;
    void *proj = base + L.proj;
    double *part = D(L.part), *sc = D(L.sc), *red = D(L.red);
    psd_info *pinfo = reinterpret_cast<psd_info *>(base + L.pinfo);
    int *sticky = reinterpret_cast<int *>(base + L.sticky);
    const int d = L.d, n = L.n;
    const int64_t nx = L.nx, ny = L.ny, nq = L.nq;
    const double gamma = 1.0 / (double)(d * d);
    const double alpha = s->alpha;

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

    // ---- setup: c = A^T G, norms, sigma, M^-1 h, eta --------------------
    SCS_TRY(psd_constraint_adjoint(d, g, cv, aff, L.aff_bytes, st));
    const int parts_x = std::min<int64_t>(SCS_PARTS, std::max<int64_t>(1, grid_of(nx + n)));
    hipLaunchKernelGGL(scs_setup_kernel, dim3(parts_x), dim3(SCS_BLOCK), 0, st, cv, g, nx, n, part);
    hipLaunchKernelGGL(scs_final3_kernel, dim3(1), dim3(64 * 3), 0, st, part, parts_x, red);
    SCS_LAUNCHED();
    double h3[3];
    SCS_READ(h3, red, sizeof h3);
    const double c_norm = std::sqrt(h3[0]), c_inf = h3[1], b0 = gamma * h3[2];
    const double b_norm = gamma * std::sqrt((double)n);
    const double sigma = (s->normalize && c_norm > 0.0) ? b_norm / c_norm : 1.0;
    hipLaunchKernelGGL(scs_h_kernel, dim3(grid_of(nx + ny)), dim3(SCS_BLOCK), 0, st, cv, mhx, mhy, nx, n, sigma,
                       gamma);
    hipLaunchKernelGGL(scs_diag_add_kernel, dim3(grid_of(n)), dim3(SCS_BLOCK), 0, st, mhy, n, gamma);
    SCS_LAUNCHED();
    SCS_TRY(psd_affine_step(d, mhx, mhy, mhx, mhy, aff, L.aff_bytes, st));
    hipLaunchKernelGGL(scs_dot_kernel, dim3(parts_x), dim3(SCS_BLOCK), 0, st, cv, mhx, mhy, nx, n, sigma, gamma, part);
    hipLaunchKernelGGL(scs_final3_kernel, dim3(1), dim3(64 * 3), 0, st, part, parts_x, red);
    SCS_LAUNCHED();
    double eta = 0.0;
    SCS_READ(&eta, red, sizeof eta);
    info->sigma = sigma;
    if (!std::isfinite(eta) || !std::isfinite(c_norm) || !std::isfinite(b0)) {
        info->status = PSD_ENONFINITE;
        return PSD_OK;
    }
    hipLaunchKernelGGL(scs_start_kernel, dim3(grid_of(nx + ny)), dim3(SCS_BLOCK), 0, st, x, y, sl, ux, uy, vy, sc,
                       nx, ny, sigma, s->warm_start);
    if (hipMemsetAsync(sticky, 0, sizeof(int), st) != hipSuccess) return PSD_EDEVICE;
    SCS_LAUNCHED();

    // the cone input q = u~_r - v of the current (u, v): (u_x, z_y, q_tau)
    auto cone_input = [&]() -> psd_status {
        hipLaunchKernelGGL(scs_sum_kernel, dim3(grid_of(nx + ny)), dim3(SCS_BLOCK), 0, st, ux, uy, vy, zx, zy, nx, ny);
        if (hipGetLastError() != hipSuccess) return PSD_EDEVICE;
        const psd_status e = psd_affine_step(d, zx, zy, zx, zy, aff, L.aff_bytes, st);
        if (e != PSD_OK) return e;
        hipLaunchKernelGGL(scs_dot_kernel, dim3(parts_x), dim3(SCS_BLOCK), 0, st, cv, zx, zy, nx, n, sigma, gamma,
                           part);
        hipLaunchKernelGGL(scs_tau_kernel, dim3(1), dim3(64), 0, st, part, parts_x, sc, eta, alpha);
        hipLaunchKernelGGL(scs_update_kernel, dim3(grid_of(nx + ny)), dim3(SCS_BLOCK), 0, st, zx, zy, mhx, mhy, ux,
                           uy, vy, sc, nx, ny, alpha);
        return hipGetLastError() == hipSuccess ? PSD_OK : PSD_EDEVICE;
    };

    // Anderson state
    const QView qv{ux, zy, sc, nx, ny};
    double *qk = L.m ? D(L.qk) : nullptr, *qprev = L.m ? D(L.qprev) : nullptr;
    double *fprev = L.m ? D(L.fprev) : nullptr, *gsave = L.m ? D(L.gsave) : nullptr;
    double *Sb = L.m ? D(L.S) : nullptr, *Yb = L.m ? D(L.Y) : nullptr;
    double *aapart = L.m ? D(L.aapart) : nullptr, *aaout = L.m ? D(L.aaout) : nullptr;
    const int aa_parts = std::min<int64_t>(SCS_PARTS, std::max<int64_t>(1, grid_of(nq)));
    AaHost aa;
    aa.m = L.m;

    // after G(q_k) is in q: the next input (accelerated, plain or restored)
    auto anderson = [&]() -> psd_status {
        int jnew = -1;
        int evict = -1;
        if (aa.have_prev) {
            if (aa.count < aa.m) {
                bool used[AA_MAX] = {};
                for (int c = 0; c < aa.count; ++c) used[aa.order[c]] = true;
                for (int i = 0; i < aa.m; ++i)
                    if (!used[i]) { jnew = i; break; }
            } else {
                jnew = evict = aa.order[0];
            }
        }
        hipLaunchKernelGGL(aa_pair_kernel, dim3(grid_of(nq)), dim3(SCS_BLOCK), 0, st, qv, qk, qprev, fprev, Sb, Yb,
                           L.ld, jnew, nq);
        AaCols cols{};
        int ncols = 0;
        for (int c = 0; c < aa.count; ++c)
            if (aa.order[c] != evict) cols.slot[ncols++] = aa.order[c];
        if (jnew >= 0) cols.slot[ncols++] = jnew;
        cols.count = ncols;
        cols.jnew = jnew;
        hipLaunchKernelGGL(aa_dot_kernel, dim3(aa_parts), dim3(SCS_BLOCK), 0, st, Sb, Yb, L.ld, fprev, cols, nq, aapart,
                           SCS_PARTS);
        const int nvals = 3 + 3 * ncols;
        hipLaunchKernelGGL(aa_dot_final_kernel, dim3(nvals), dim3(64), 0, st, aapart, aa_parts, SCS_PARTS, aaout);
        if (hipGetLastError() != hipSuccess) return PSD_EDEVICE;
        double v[AA_VALS];
        if (hipMemcpyAsync(v, aaout, sizeof(double) * nvals, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return PSD_EDEVICE;
        const double nf = std::sqrt(v[0]);
        if (aa.pending) {
            aa.pending = false;
            if (!(nf <= 2.0 * aa.nf_save)) {      // safeguard: back to the plain input
                hipLaunchKernelGGL(aa_copy_kernel, dim3(grid_of(nq)), dim3(SCS_BLOCK), 0, st, qv, qk, gsave, nq);
                aa.reset();
                ++aa.rejected;
                return hipGetLastError() == hipSuccess ? PSD_OK : PSD_EDEVICE;
            }
        }
        if (jnew >= 0) {
            for (int c = 0; c < ncols; ++c) {
                const int i = cols.slot[c];
                aa.M[i][jnew] = v[3 + 3 * c];   // s_i^T y_j
                aa.M[jnew][i] = v[4 + 3 * c];   // s_j^T y_i
            }
            aa.ss[jnew] = v[1];
            aa.yy[jnew] = v[2];
            for (int c = 0; c < ncols; ++c) aa.order[c] = cols.slot[c];
            aa.count = ncols;
        }
        aa.have_prev = true;
        bool step = aa.count > 0;
        AaGamma gm{};
        if (step) {
            const int c = aa.count;
            double A[AA_MAX * AA_MAX], b[AA_MAX], s2 = 0.0, y2 = 0.0;
            for (int p = 0; p < c; ++p) {
                s2 += aa.ss[aa.order[p]];
                y2 += aa.yy[aa.order[p]];
            }
            const double lam = 1e-8 * std::sqrt(s2) * std::sqrt(y2);
            for (int p = 0; p < c; ++p) {
                for (int q2 = 0; q2 < c; ++q2) A[p * c + q2] = aa.M[aa.order[p]][aa.order[q2]] + (p == q2 ? lam : 0.0);
                b[p] = v[5 + 3 * p];              // s_i^T f, columns in the order above
            }
            step = small_solve(c, A, b);
            for (int p = 0; step && p < c; ++p) step = std::fabs(b[p]) <= 1e10;
            if (step) {
                for (int p = 0; p < c; ++p) {
                    gm.g[p] = b[p];
                    gm.slot[p] = aa.order[p];
                }
                gm.count = c;
            }
        }
        if (step) {
            hipLaunchKernelGGL(aa_extrapolate_kernel, dim3(grid_of(nq)), dim3(SCS_BLOCK), 0, st, qv, Sb, Yb, L.ld, gm,
                               qk, gsave, nq);
            aa.pending = true;
            aa.nf_save = nf;
            ++aa.accepted;
        } else {
            hipLaunchKernelGGL(aa_copy_kernel, dim3(grid_of(nq)), dim3(SCS_BLOCK), 0, st, qv, qk, nullptr, nq);
        }
        return hipGetLastError() == hipSuccess ? PSD_OK : PSD_EDEVICE;
    };

    // ---- iterations -------------------------------------------------------
    const int parts_r = std::min(SCS_PARTS, std::max(n, 1));
    const double bound_b = gamma;   // ||b||_inf
    int status = PSD_ENOCONV;
    int k = 0;
    bool switched = false;   // left the mixed cone steps on the residuals
    double r[R_SLOTS + 2] = {};
    SCS_TRY(cone_input());
    if (L.m) {
        hipLaunchKernelGGL(aa_copy_kernel, dim3(grid_of(nq)), dim3(SCS_BLOCK), 0, st, qv, qk, nullptr, nq);
        SCS_LAUNCHED();
    }
    for (k = 1; k <= s->max_iters; ++k) {
        // cone step: u_y = Pi(q_y), v_s = u_y - q_y, tau, kappa
        const psd_mode mode = (k <= s->mixed_iters && !switched) ? (psd_mode)s->mixed_mode : PSD_FP64_EIG;
        SCS_TRY(psd_project(n, zy, uy, mode, proj, L.proj_bytes, st, pinfo, nullptr));
        hipLaunchKernelGGL(scs_fold_kernel, dim3(1), dim3(64), 0, st, pinfo, sticky);
        hipLaunchKernelGGL(scs_dual_kernel, dim3(grid_of(ny)), dim3(SCS_BLOCK), 0, st, vy, zy, uy, sc, ny);
        SCS_LAUNCHED();
        if (k % s->check_every == 0 || k == s->max_iters) {
            SCS_TRY(psd_constraint_apply(d, ux, ty, aff, L.aff_bytes, st));
            SCS_TRY(psd_constraint_adjoint(d, uy, tx, aff, L.aff_bytes, st));
            hipLaunchKernelGGL(scs_resid_kernel, dim3(parts_r), dim3(SCS_BLOCK), 0, st, ty, vy, uy, tx, ux, cv, sc, n,
                               nx, sigma, gamma, part);
            hipLaunchKernelGGL(scs_resid_final_kernel, dim3(1), dim3(64 * R_SLOTS), 0, st, part, parts_r, sc, red);
            SCS_LAUNCHED();
            SCS_READ(r, red, sizeof r);
            const double tau = r[R_SLOTS], kappa = r[R_SLOTS + 1];
            info->tau = tau;
            info->kappa = kappa;
            bool finite = std::isfinite(tau) && std::isfinite(kappa);
            for (int q2 = 0; q2 < R_SLOTS; ++q2) finite = finite && std::isfinite(r[q2]);
            if (!finite) {
                status = PSD_ENONFINITE;
                break;
            }
            if (tau > 0.0) {
                const double it = 1.0 / tau, ist = 1.0 / (sigma * tau);
                const double res_pri = r[R_PRI] * it, ax_inf = r[R_AX] * it, s_inf = r[R_S] * it;
                const double res_dual = r[R_DUAL] * ist, aty_inf = r[R_ATY] * ist;
                const double cx = r[R_CX] * it, by = gamma * r[R_TRY] * ist;
                const double gap = std::fabs(cx + by);
                info->res_pri = res_pri;
                info->res_dual = res_dual;
                info->gap = gap;
                info->pobj = b0 - cx;
                info->dobj = b0 + by;
                const double e = s->eps;
                const double bp = e + e * std::max(ax_inf, std::max(s_inf, bound_b));
                const double bd = e + e * std::max(aty_inf, c_inf);
                const double bg = e + e * std::max(std::fabs(cx), std::fabs(by));
                if (e > 0.0 && res_pri <= bp && res_dual <= bd && gap <= bg) {
                    status = PSD_OK;
                    break;
                }
                const double ms = s->mixed_switch;
                if (ms > 0.0 && e > 0.0 && k <= s->mixed_iters && !switched && res_pri <= ms * bp &&
                    res_dual <= ms * bd && gap <= ms * bg) {
                    switched = true;
                    info->switch_iter = k;
                }
            } else {
                info->res_pri = info->res_dual = info->gap = INFINITY;
            }
        }
        if (k == s->max_iters) break;
        SCS_TRY(cone_input());
        if (L.m) SCS_TRY(anderson());
    }
    info->iters = std::min(k, s->max_iters);
    info->aa_accepted = aa.accepted;
    info->aa_rejected = aa.rejected;
    int proj_status = 0;
    SCS_READ(&proj_status, sticky, sizeof proj_status);
    info->proj_status = proj_status;
    if (status == PSD_OK && proj_status == PSD_ENONFINITE) status = PSD_ENONFINITE;

    hipLaunchKernelGGL(scs_out_kernel, dim3(grid_of(nx + ny)), dim3(SCS_BLOCK), 0, st, ux, uy, vy, x, y, sl, sc, nx,
                       ny, sigma);
    SCS_LAUNCHED();

    // ---- post-processing of W = b - A x (App. "Sparse SDP formulation") --
    if (w && info->tau > 0.0 && status != PSD_ENONFINITE) {
        SCS_TRY(psd_constraint_apply(d, ux, ty, aff, L.aff_bytes, st));
        hipLaunchKernelGGL(scs_scale_kernel, dim3(grid_of(ny)), dim3(SCS_BLOCK), 0, st, ty, w, sc, ny, -1.0, 1);
        hipLaunchKernelGGL(scs_diag_add_kernel, dim3(grid_of(n)), dim3(SCS_BLOCK), 0, st, w, n, gamma);
        SCS_LAUNCHED();
        // lambda_min(W) from the saved eigenvalues (ascending) of an FP64 projection
        double *saved = static_cast<double *>(aff);
        SCS_TRY(psd_project(n, w, zy, PSD_FP64_EIG, proj, L.proj_bytes, st, pinfo, saved));
        double lmin = 0.0;
        psd_info pi{};
        if (hipMemcpyAsync(&lmin, saved, sizeof lmin, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&pi, pinfo, sizeof pi, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return PSD_EDEVICE;
        double lam = 0.0;
        if (pi.status == PSD_OK && lmin < 0.0) {
            lam = -lmin / (gamma - lmin);
            hipLaunchKernelGGL(scs_scale_kernel, dim3(grid_of(ny)), dim3(SCS_BLOCK), 0, st, w, w, sc, ny, 1.0 - lam, 0);
            hipLaunchKernelGGL(scs_diag_add_kernel, dim3(grid_of(n)), dim3(SCS_BLOCK), 0, st, w, n, lam * gamma);
            SCS_LAUNCHED();
        }
        info->post_lambda = lam;
        info->post_lambda_min = lmin;
    }
    info->status = status;
#undef SCS_TRY
#undef SCS_LAUNCHED
#undef SCS_READ
    return PSD_OK;
}

}  // extern "C"
