/*
 * psd_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU reference for the Euclidean projection
 * onto the cone of complex Hermitian positive-semidefinite matrices, as used in
 * the cone step of the SCS iteration (App. D.1, eq. final_iterates2), and for
 * its derivative.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code with the GPU
 * library: no headers, no helpers, no tables.
 *
 * What is computed, and where the paper defines it:
 *   - vec_R / mat_R (App. D.1, the real encoding of a Hermitian matrix): the
 *     diagonal entries X_ii and sqrt(2) Re X_ij, sqrt(2) Im X_ij for i<j.  The
 *     paper leaves the ordering open; this file fixes it as row-major over the
 *     upper triangle: row i holds X_ii, then the (Re, Im) pairs of X_ij for
 *     j = i+1..n-1.  Row i therefore starts at offset i*(2n-i).
 *   - Pi(X): the Euclidean projection onto the PSD cone (App. D.1, Pi_S), which
 *     App. D.2 implements as an eigendecomposition with the negative
 *     eigenvalues set to zero: Pi(X) = V diag(max(lambda,0)) V^H.  The
 *     eigendecomposition here is the textbook cyclic complex Jacobi method
 *     (a 2x2 phase to make the pivot real, then a real symmetric Jacobi
 *     rotation), either in row-cyclic order or in round-robin (tournament)
 *     order whose n/2 disjoint rotations per round are applied together.
 *     The reconstruction is accumulated in long double.
 *   - The derivative DPi(X)[E] (needed to back-propagate through the
 *     projection, App. E): the Daleckii-Krein formula
 *       DPi(X)[E] = V (Gamma o (V^H E V)) V^H,
 *     Gamma_ij the divided difference of f(t)=max(t,0) at (lambda_i, lambda_j),
 *     with f'(0) taken as 0.  DPi(X) is self-adjoint, so this is also the VJP.
 *
 * Matrices are row-major n x n arrays of double complex.
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 3
#define OR_ENOCONV 5

#define OR_MAX_SWEEPS 60

/* ------------------------------------------------------------------------- */
/* vec_R and mat_R (App. D.1)                                                 */
/* ------------------------------------------------------------------------- */

long or_svec_row_offset(int n, int i) { return (long)i * (2L * n - i); }

/* Index of sqrt2*Re X_ij (i<j) in the svec; Im follows at +1. */
long or_svec_offdiag_offset(int n, int i, int j) {
    return or_svec_row_offset(n, i) + 1 + 2L * (j - i - 1);
}

int or_unpack(int n, const double *s, cplx *a) {
    if (n < 1 || !s || !a) return OR_EINVAL;
    for (int i = 0; i < n; ++i) {
        a[(long)i * n + i] = s[or_svec_row_offset(n, i)];
        for (int j = i + 1; j < n; ++j) {
            long o = or_svec_offdiag_offset(n, i, j);
            double re = s[o] / M_SQRT2, im = s[o + 1] / M_SQRT2;
            a[(long)i * n + j] = re + im * I;
            a[(long)j * n + i] = re - im * I;
        }
    }
    return OR_OK;
}

/* Packs the upper triangle; the imaginary part of the diagonal is dropped. */
int or_pack(int n, const cplx *a, double *s) {
    if (n < 1 || !s || !a) return OR_EINVAL;
    for (int i = 0; i < n; ++i) {
        s[or_svec_row_offset(n, i)] = creal(a[(long)i * n + i]);
        for (int j = i + 1; j < n; ++j) {
            long o = or_svec_offdiag_offset(n, i, j);
            s[o] = M_SQRT2 * creal(a[(long)i * n + j]);
            s[o + 1] = M_SQRT2 * cimag(a[(long)i * n + j]);
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Complex cyclic Jacobi eigendecomposition                                   */
/* ------------------------------------------------------------------------- */

/* Parameters of the unitary G acting on coordinates (p,q) that diagonalises
 * the 2x2 Hermitian block [[app, apq], [conj(apq), aqq]]:
 *   G = diag(1, e^{-i phi}) * [[c, s], [-s, c]],  apq = r e^{i phi}.
 * The phase makes the pivot real (= r); the real rotation is the symmetric
 * Schur decomposition of [[app, r], [r, aqq]]:
 *   tau = (aqq - app)/(2r), t = sgn(tau)/(|tau| + sqrt(1+tau^2)), sgn(0)=1,
 *   c = 1/sqrt(1+t^2), s = t c; new diagonal app - t r, aqq + t r. */
typedef struct {
    int p, q, active;
    double c, s, r, t;
    cplx ph; /* e^{-i phi} */
} rot_t;

static int or_rot_params(const cplx *a, int n, int p, int q, double tiny, rot_t *g) {
    cplx apq = a[(long)p * n + q];
    double app = creal(a[(long)p * n + p]), aqq = creal(a[(long)q * n + q]);
    double r = cabs(apq);
    g->p = p; g->q = q; g->active = 0;
    /* Skip negligible pivots: relative to the diagonal (high relative
       accuracy) or, below an absolute floor, relative to ||A||_F. */
    if (r == 0.0 || r <= DBL_EPSILON * sqrt(fabs(app) * fabs(aqq)) || r <= tiny) return 0;
    double tau = (aqq - app) / (2.0 * r);
    double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    double c = 1.0 / sqrt(1.0 + t * t);
    g->c = c; g->s = t * c; g->r = r; g->t = t;
    g->ph = conj(apq) / r;
    g->active = 1;
    return 1;
}

/* A <- A G on columns p,q (rows lo..hi-1); likewise used for V. */
static void or_rot_cols(cplx *a, int n, const rot_t *g, int lo, int hi) {
    const int p = g->p, q = g->q;
    const cplx gqp = -g->s * g->ph, gqq = g->c * g->ph;
    for (int k = lo; k < hi; ++k) {
        cplx xp = a[(long)k * n + p], xq = a[(long)k * n + q];
        a[(long)k * n + p] = g->c * xp + gqp * xq;
        a[(long)k * n + q] = g->s * xp + gqq * xq;
    }
}

/* A <- G^H A on rows p,q (columns lo..hi-1). */
static void or_rot_rows(cplx *a, int n, const rot_t *g, int lo, int hi) {
    const int p = g->p, q = g->q;
    const cplx hqp = -g->s * conj(g->ph), hqq = g->c * conj(g->ph);
    for (int k = lo; k < hi; ++k) {
        cplx xp = a[(long)p * n + k], xq = a[(long)q * n + k];
        a[(long)p * n + k] = g->c * xp + hqp * xq;
        a[(long)q * n + k] = g->s * xp + hqq * xq;
    }
}

/* The (p,q) block of G^H A G is diag(app - t r, aqq + t r) in exact
   arithmetic; store that exactly. */
static void or_rot_finish(cplx *a, int n, const rot_t *g, double app, double aqq) {
    a[(long)g->p * n + g->p] = app - g->t * g->r;
    a[(long)g->q * n + g->q] = aqq + g->t * g->r;
    a[(long)g->p * n + g->q] = 0.0;
    a[(long)g->q * n + g->p] = 0.0;
}

static double or_frob(const cplx *a, long nn) {
    long double s = 0.0L;
    for (long k = 0; k < nn; ++k) s += (long double)creal(a[k]) * creal(a[k]) + (long double)cimag(a[k]) * cimag(a[k]);
    return (double)sqrtl(s);
}

/* Row-cyclic sweeps: (0,1),(0,2),...,(0,n-1),(1,2),... one rotation at a time. */
static int or_jacobi_serial(int n, cplx *a, cplx *v, double tiny, int max_sweeps,
                            int *sweeps, long *rotations) {
    for (int sw = 0; sw < max_sweeps; ++sw) {
        long nrot = 0;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                rot_t g;
                double app = creal(a[(long)p * n + p]), aqq = creal(a[(long)q * n + q]);
                if (!or_rot_params(a, n, p, q, tiny, &g)) continue;
                or_rot_cols(a, n, &g, 0, n);
                or_rot_rows(a, n, &g, 0, n);
                or_rot_finish(a, n, &g, app, aqq);
                or_rot_cols(v, n, &g, 0, n);
                ++nrot;
            }
        *rotations += nrot;
        *sweeps = sw + 1;
        if (nrot == 0) return OR_OK;
    }
    return OR_ENOCONV;
}

/* Round-robin (circle-method) ordering: m = n rounded up to even players;
   in round r player 0 stays, the others rotate; pairs are (pos k, pos m-1-k).
   Each round's pairs are disjoint, so all their rotations commute: compute
   every parameter from the current A, apply all column rotations, then all row
   rotations.  The result does not depend on the thread count. */
static int or_rr_player(int pos, int r, int m) { return pos == 0 ? 0 : 1 + (pos - 1 + r) % (m - 1); }

static int or_jacobi_roundrobin(int n, cplx *a, cplx *v, double tiny, int max_sweeps,
                                int *sweeps, long *rotations) {
    const int m = n + (n & 1);
    const int npair = m / 2;
    rot_t *g = (rot_t *)malloc(sizeof(rot_t) * npair);
    double *dg = (double *)malloc(sizeof(double) * 2 * npair);
    if (!g || !dg) { free(g); free(dg); return OR_ENOMEM; }
    int status = OR_ENOCONV;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        long nrot = 0;
        for (int r = 0; r < m - 1; ++r) {
            int nact = 0;
            for (int k = 0; k < npair; ++k) {
                int x = or_rr_player(k, r, m), y = or_rr_player(m - 1 - k, r, m);
                int p = x < y ? x : y, q = x < y ? y : x;
                g[k].active = 0;
                if (q >= n) continue; /* the dummy player of odd n */
                dg[2 * k] = creal(a[(long)p * n + p]);
                dg[2 * k + 1] = creal(a[(long)q * n + q]);
                nact += or_rot_params(a, n, p, q, tiny, &g[k]);
            }
            if (!nact) continue;
            nrot += nact;
#pragma omp parallel for schedule(static)
            for (int k = 0; k < npair; ++k)
                if (g[k].active) { or_rot_cols(a, n, &g[k], 0, n); or_rot_cols(v, n, &g[k], 0, n); }
#pragma omp parallel for schedule(static)
            for (int k = 0; k < npair; ++k)
                if (g[k].active) or_rot_rows(a, n, &g[k], 0, n);
            for (int k = 0; k < npair; ++k)
                if (g[k].active) or_rot_finish(a, n, &g[k], dg[2 * k], dg[2 * k + 1]);
        }
        *rotations += nrot;
        *sweeps = sw + 1;
        if (nrot == 0) { status = OR_OK; break; }
    }
    free(g); free(dg);
    return status;
}

/* Eigendecomposition A = V diag(lam) V^H of the Hermitian matrix in `a`
   (overwritten: it ends up diagonal).  v: n*n row-major, column k is the
   eigenvector of lam[k].  Eigenvalues are returned unsorted (Jacobi order),
   with `order` (nullable) receiving the ascending permutation. */
int or_jacobi(int n, cplx *a, cplx *v, double *lam, int mode, int max_sweeps,
              int *sweeps, long *rotations) {
    if (n < 1 || !a || !v || !lam) return OR_EINVAL;
    int sw = 0; long rot = 0;
    if (max_sweeps <= 0) max_sweeps = OR_MAX_SWEEPS;
    /* Hermitian input: force the diagonal real. */
    for (int i = 0; i < n; ++i) a[(long)i * n + i] = creal(a[(long)i * n + i]);
    for (long k = 0; k < (long)n * n; ++k) v[k] = 0.0;
    for (int i = 0; i < n; ++i) v[(long)i * n + i] = 1.0;
    const double tiny = DBL_EPSILON * DBL_EPSILON * or_frob(a, (long)n * n);
    int st = mode == 0 ? or_jacobi_serial(n, a, v, tiny, max_sweeps, &sw, &rot)
                       : or_jacobi_roundrobin(n, a, v, tiny, max_sweeps, &sw, &rot);
    for (int i = 0; i < n; ++i) lam[i] = creal(a[(long)i * n + i]);
    if (sweeps) *sweeps = sw;
    if (rotations) *rotations = rot;
    return st;
}

/* ------------------------------------------------------------------------- */
/* Projection and its derivative                                             */
/* ------------------------------------------------------------------------- */

/* Eigendecomposition of mat_R(x): lam (n), v (n*n complex, row-major). */
int or_eigh_svec(int n, const double *x, double *lam, cplx *v, int mode, int max_sweeps,
                 int *sweeps, long *rotations) {
    if (n < 1 || !x || !lam || !v) return OR_EINVAL;
    cplx *a = (cplx *)malloc(sizeof(cplx) * (size_t)n * n);
    if (!a) return OR_ENOMEM;
    or_unpack(n, x, a);
    int st = or_jacobi(n, a, v, lam, mode, max_sweeps, sweeps, rotations);
    free(a);
    return st;
}

/* Pi = V diag(max(lam,0)) V^H accumulated in long double, packed to svec. */
int or_reconstruct(int n, const double *lam, const cplx *v, double *y) {
    if (n < 1 || !lam || !v || !y) return OR_EINVAL;
    cplx *pm = (cplx *)malloc(sizeof(cplx) * (size_t)n * n);
    if (!pm) return OR_ENOMEM;
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < n; ++i)
        for (int j = i; j < n; ++j) {
            long double re = 0.0L, im = 0.0L;
            for (int k = 0; k < n; ++k) {
                if (!(lam[k] > 0.0)) continue;
                /* V_ik * lam_k * conj(V_jk) */
                long double ar = creal(v[(long)i * n + k]), ai = cimag(v[(long)i * n + k]);
                long double br = creal(v[(long)j * n + k]), bi = cimag(v[(long)j * n + k]);
                re += (long double)lam[k] * (ar * br + ai * bi);
                im += (long double)lam[k] * (ai * br - ar * bi);
            }
            pm[(long)i * n + j] = (double)re + (double)im * I;
            pm[(long)j * n + i] = (double)re - (double)im * I;
        }
    or_pack(n, pm, y);
    free(pm);
    return OR_OK;
}

/* y = svec(Pi(mat(x))).  lam_out (n) and v_out (n*n complex) are optional. */
int or_project(int n, const double *x, double *y, int mode, int *sweeps,
               double *lam_out, cplx *v_out) {
    if (n < 1 || !x || !y) return OR_EINVAL;
    double *lam = (double *)malloc(sizeof(double) * n);
    cplx *v = (cplx *)malloc(sizeof(cplx) * (size_t)n * n);
    if (!lam || !v) { free(lam); free(v); return OR_ENOMEM; }
    long rot = 0;
    int st = or_eigh_svec(n, x, lam, v, mode, 0, sweeps, &rot);
    if (st == OR_OK) st = or_reconstruct(n, lam, v, y);
    if (lam_out) memcpy(lam_out, lam, sizeof(double) * n);
    if (v_out) memcpy(v_out, v, sizeof(cplx) * (size_t)n * n);
    free(lam); free(v);
    return st;
}

/* Divided difference of f(t) = max(t,0) at (a, b), with f'(0) := 0:
   1 if both positive, 0 if both non-positive, a/(a-b) if a > 0 >= b. */
static double or_gamma(double a, double b) {
    int pa = a > 0.0, pb = b > 0.0;
    if (pa && pb) return 1.0;
    if (!pa && !pb) return 0.0;
    return pa ? a / (a - b) : b / (b - a);
}

/* gx = svec(V (Gamma o (V^H G V)) V^H), G = mat(gy); DK formula. */
int or_vjp(int n, const double *x, const double *gy, double *gx, int mode) {
    if (n < 1 || !x || !gy || !gx) return OR_EINVAL;
    size_t nn = (size_t)n * n;
    double *lam = (double *)malloc(sizeof(double) * n);
    cplx *v = (cplx *)malloc(sizeof(cplx) * nn);
    cplx *g = (cplx *)malloc(sizeof(cplx) * nn);
    cplx *t = (cplx *)malloc(sizeof(cplx) * nn);
    cplx *m = (cplx *)malloc(sizeof(cplx) * nn);
    int st = OR_ENOMEM;
    if (!lam || !v || !g || !t || !m) goto out;
    long rot = 0; int sw = 0;
    st = or_eigh_svec(n, x, lam, v, mode, 0, &sw, &rot);
    if (st != OR_OK) goto out;
    or_unpack(n, gy, g);
    /* t = G V */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            cplx s = 0.0;
            for (int k = 0; k < n; ++k) s += g[(long)i * n + k] * v[(long)k * n + j];
            t[(long)i * n + j] = s;
        }
    /* m = Gamma o (V^H t) */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            cplx s = 0.0;
            for (int k = 0; k < n; ++k) s += conj(v[(long)k * n + i]) * t[(long)k * n + j];
            m[(long)i * n + j] = or_gamma(lam[i], lam[j]) * s;
        }
    /* t = m V^H */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            cplx s = 0.0;
            for (int k = 0; k < n; ++k) s += m[(long)i * n + k] * conj(v[(long)j * n + k]);
            t[(long)i * n + j] = s;
        }
    /* g = V t */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            cplx s = 0.0;
            for (int k = 0; k < n; ++k) s += v[(long)i * n + k] * t[(long)k * n + j];
            g[(long)i * n + j] = s;
        }
    or_pack(n, g, gx);
out:
    free(lam); free(v); free(g); free(t); free(m);
    return st;
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
