/* Host memory and undefined-behaviour check of the oracle (test
 * infrastructure): built by tests/test_oracle_asan.py with gcc's address and
 * undefined-behaviour sanitizers and run on small orders in both Jacobi
 * orderings.  Inputs come from a plain linear congruential generator; the
 * checks are the projection's own identities (Moreau: Pi(X) - Pi(-X) = X;
 * idempotence: Pi(Pi(X)) = Pi(X)), the derivative's Euler identity
 * DPi(X)[X] = Pi(X), and the pack/unpack round trip.  Prints "ok" and exits
 * 0 when every call succeeds and every identity holds to 1e-10. */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex cplx;
int or_unpack(int n, const double *s, cplx *a);
int or_pack(int n, const cplx *a, double *s);
int or_project(int n, const double *x, double *y, int mode, int *sweeps, double *lam_out, cplx *v_out);
int or_vjp(int n, const double *x, const double *gy, double *gx, int mode);

static unsigned long long state = 88172645463325252ULL;
static double next_unit(void) {
    state = state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

static double rel(const double *a, const double *b, long m) {
    double d = 0.0, r = 0.0;
    for (long i = 0; i < m; ++i) {
        d += (a[i] - b[i]) * (a[i] - b[i]);
        r += b[i] * b[i];
    }
    return sqrt(d) / (r > 0.0 ? sqrt(r) : 1.0);
}

int main(void) {
    const int orders[] = {1, 2, 3, 7, 16, 33};
    int bad = 0;
    for (unsigned k = 0; k < sizeof orders / sizeof orders[0]; ++k) {
        const int n = orders[k];
        const long m = (long)n * n;
        double *x = malloc(sizeof(double) * m), *xn = malloc(sizeof(double) * m);
        double *y = malloc(sizeof(double) * m), *yn = malloc(sizeof(double) * m);
        double *yy = malloc(sizeof(double) * m), *g = malloc(sizeof(double) * m);
        double *s = malloc(sizeof(double) * m);
        cplx *a = malloc(sizeof(cplx) * m);
        for (long i = 0; i < m; ++i) {
            x[i] = next_unit();
            xn[i] = -x[i];
        }
        for (int mode = 0; mode < 2; ++mode) {
            int sw = 0;
            if (or_project(n, x, y, mode, &sw, NULL, NULL) || or_project(n, xn, yn, mode, &sw, NULL, NULL) ||
                or_project(n, y, yy, mode, &sw, NULL, NULL) || or_vjp(n, x, x, g, mode)) {
                ++bad;
                continue;
            }
            for (long i = 0; i < m; ++i) s[i] = y[i] - yn[i];
            const double e1 = rel(s, x, m), e2 = rel(yy, y, m), e3 = rel(g, y, m);
            if (e1 > 1e-10 || e2 > 1e-10 || e3 > 1e-10) {
                printf("n=%d mode=%d: Moreau %.2e, idempotence %.2e, Euler %.2e\n", n, mode, e1, e2, e3);
                ++bad;
            }
        }
        /* off-diagonal entries are divided by sqrt2 and multiplied back: a
           round trip to rounding */
        if (or_unpack(n, x, a) || or_pack(n, a, s) || rel(s, x, m) > 1e-15) {
            printf("n=%d: pack/unpack %.2e\n", n, rel(s, x, m));
            ++bad;
        }
        free(x); free(xn); free(y); free(yn); free(yy); free(g); free(s); free(a);
    }
    if (bad) {
        printf("%d failures\n", bad);
        return 1;
    }
    printf("ok\n");
    return 0;
}
