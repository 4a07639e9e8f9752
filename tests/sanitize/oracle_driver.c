/* Runs the CPU oracle on small grids in each of its modes (both schemes,
 * Newton and Picard, Neumann axes, pinning, sides that are not powers of two,
 * dense Newton, three dimensions), for the sanitizer build of the oracle
 * (tests/test_sanitizers_cpu.py).  Exit status 0 and "oracle driver ok" when
 * every step returns a cycle count and finite results. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int scheme;
    double h, s, M, beta, eps;
} orc_model;

void orc_set_bc(int neumann_x, int neumann_y);
int orc_step(const orc_model *p, int newton, int m, int n, const double *phik,
             const double *phikm1, const double *psik, int guess, int nu1, int nu2, int coarsest,
             int coarse_sweeps, double tol, int max_cycles, double *phinew, double *mu,
             double *ka, double *psinew, double *history, double *energies, const double *pin,
             const double *phihat);
int o3_step(int scheme, int newton, int m, int n, int l, double h, double s, double M,
            double beta, double eps, const double *phik, const double *phikm1,
            const double *psik, int guess, int nu1, int nu2, int coarsest, int coarse_sweeps,
            double tol, int max_cycles, double *phinew, double *mu, double *ka,
            double *psinew, double *history, double *energies);

static double frand(unsigned *state) {
    *state = *state * 1664525u + 1013904223u;
    return (double)(*state >> 8) / 16777216.0;
}

static int check(const char *what, int cyc, const double *a, size_t n) {
    for (size_t q = 0; q < n; ++q)
        if (!isfinite(a[q])) {
            printf("%s: non-finite value\n", what);
            return 1;
        }
    if (cyc < 0) {
        printf("%s: not converged (%d)\n", what, cyc);
        return 1;
    }
    return 0;
}

static int step2(const char *what, int scheme, int newton, int m, int n, int bcx, int bcy,
                 int pinned, int coarse_sweeps) {
    size_t N = (size_t)m * n;
    double *buf = calloc(12 * N + 256, sizeof(double));
    double *phik = buf, *phikm1 = buf + N, *psik = buf + 2 * N, *phinew = buf + 3 * N;
    double *mu = buf + 4 * N, *ka = buf + 5 * N, *psinew = buf + 6 * N, *pin = buf + 7 * N;
    double *hat = buf + 8 * N, *hist = buf + 12 * N, en[4];
    unsigned st = 12345u + (unsigned)(m * 31 + n);
    for (size_t q = 0; q < N; ++q) {
        phik[q] = 0.1 + 0.1 * (frand(&st) - 0.5);
        phikm1[q] = phik[q] + 0.001 * (frand(&st) - 0.5);
        psik[q] = 0.01 * (frand(&st) - 0.5);
        pin[q] = (q < (size_t)m) ? 2.0 : 0.0;
        hat[q] = phik[q];
    }
    orc_model p = {scheme, 0.5, 0.1, 1.0, 0.9, 0.025};
    orc_set_bc(bcx, bcy);
    int cyc = orc_step(&p, newton, m, n, phik, phikm1, psik, 1, 2, 2, 2, coarse_sweeps, 1e-11,
                       200, phinew, mu, ka, psinew, hist, en, pinned ? pin : NULL,
                       pinned ? hat : NULL);
    orc_set_bc(0, 0);
    int rc = check(what, cyc, phinew, N) || check(what, cyc, en, 4);
    free(buf);
    return rc;
}

int main(void) {
    int bad = 0;
    bad |= step2("scheme 1 Newton 16x16", 1, 1, 16, 16, 0, 0, 0, 0);
    bad |= step2("scheme 1 Picard 16x16", 1, 0, 16, 16, 0, 0, 0, 0);
    bad |= step2("scheme 2 Newton 16x16", 2, 1, 16, 16, 0, 0, 0, 0);
    bad |= step2("scheme 2 Picard 16x32", 2, 0, 16, 32, 0, 0, 0, 0);
    bad |= step2("scheme 2 Neumann y 16x16", 2, 1, 16, 16, 0, 1, 0, 0);
    bad |= step2("scheme 2 Neumann xy 32x16", 2, 1, 32, 16, 1, 1, 0, 0);
    bad |= step2("scheme 2 pinned 16x16", 2, 1, 16, 16, 0, 0, 1, 0);
    bad |= step2("scheme 2 general 24x20", 2, 1, 24, 20, 0, 0, 0, 2);
    bad |= step2("scheme 1 dense coarsest 4x4", 1, 1, 4, 4, 0, 0, 0, 0);
    {
        int m = 8, n = 8, l = 8;
        size_t N = (size_t)m * n * l;
        double *buf = calloc(8 * N + 256, sizeof(double));
        double *phik = buf, *phinew = buf + N, *mu = buf + 2 * N, *ka = buf + 3 * N;
        double *psik = buf + 4 * N, *psinew = buf + 5 * N, *hist = buf + 6 * N, en[4];
        unsigned st = 777u;
        for (size_t q = 0; q < N; ++q) phik[q] = 0.07 + 0.05 * (frand(&st) - 0.5);
        int cyc = o3_step(2, 1, m, n, l, 0.785, 0.05, 1.0, 0.9, 0.025, phik, phik, psik, 1, 2, 2,
                          2, 2, 1e-11, 200, phinew, mu, ka, psinew, hist, en);
        bad |= check("three dimensions 8^3", cyc, phinew, N);
        free(buf);
    }
    if (bad) return 1;
    printf("oracle driver ok\n");
    return 0;
}
