/*
 * CPU oracle, three space dimensions (TEST INFRASTRUCTURE ONLY).
 *
 * The schemes of Sec. 3.1 and Sec. 3.2 and the multigrid of App. B on a
 * cell-centred m x n x l grid with spacing h, periodic in every axis.  The
 * paper works in two dimensions and states that the extension to three is
 * straightforward; this file is that extension taken literally: the
 * five-point Laplacian of App. A becomes the seven-point one,
 *   Delta_h f = (sum of the six face neighbours - 6 f) / h^2,
 * grid sums carry h^3 instead of h^2, the gradient norm sums the squared
 * differences over east, north and top cell faces times h (h^3 / h^2), the
 * restriction averages the 2 x 2 x 2 fine cells under a coarse cell and the
 * prolongation is trilinear (weights (3/4, 1/4) per axis).  Everything else
 * (equations N(u) = S of App. B.1 / B.2, the correction-form collective
 * red-black smoother with red = (i + j + k) even, the FAS V-cycle, the
 * residual norm, psi update, energies) is the two-dimensional oracle's
 * reading unchanged.  Cell (i, j, k) is stored at (k n + j) m + i.
 *
 * Plain loops, FP64, no fused multiply-add (-ffp-contract=off).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IX3(i, j, k, m, n) (((size_t)(k) * (size_t)(n) + (size_t)(j)) * (size_t)(m) + (size_t)(i))

static int wr(int i, int m) { return ((i % m) + m) % m; }

/* Sum of the six face neighbours (periodic). */
static double nsum3(const double *f, int i, int j, int k, int m, int n, int l) {
    return f[IX3(wr(i + 1, m), j, k, m, n)] + f[IX3(wr(i - 1, m), j, k, m, n)] +
           f[IX3(i, wr(j + 1, n), k, m, n)] + f[IX3(i, wr(j - 1, n), k, m, n)] +
           f[IX3(i, j, wr(k + 1, l), m, n)] + f[IX3(i, j, wr(k - 1, l), m, n)];
}

static double lap3(const double *f, int i, int j, int k, int m, int n, int l, double h) {
    return (nsum3(f, i, j, k, m, n, l) - 6.0 * f[IX3(i, j, k, m, n)]) / (h * h);
}

void o3_laplacian(int m, int n, int l, double h, const double *f, double *out) {
    for (int k = 0; k < l; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i) out[IX3(i, j, k, m, n)] = lap3(f, i, j, k, m, n, l, h);
}

/* Nonlinear term of N^(2) (App. B.1: phi^3; App. B.2: chi(phi, phi^k)(phi + phi^k)/2
 * with chi(a, b) = (a^2 + b^2)/2) and its derivative in phi. */
static double g3(int scheme, double x, double xk) {
    if (scheme == 1) return x * x * x;
    return 0.5 * (0.5 * (x * x + xk * xk)) * (x + xk);
}
static double g3p(int scheme, double x, double xk) {
    if (scheme == 1) return 3.0 * x * x;
    return (2.0 * x * (x + xk) + x * x + xk * xk) / 4.0;
}
static double al3(int scheme, double alpha) { return scheme == 1 ? alpha : 0.5 * alpha; }
static double e3(int scheme) { return scheme == 1 ? 1.0 : 0.5; }

/* Source S (App. B.1, B.2): scheme 1: S1 = phi^k + d psi^k, S2 = 2 Lap phi^k,
 * S3 = 0; scheme 2: S1 = phi^k + d psi^k, S2 = alpha/2 phi^k + 2 Lap phi~ with
 * phi~ = (3 phi^k - phi^{k-1})/2, S3 = Lap phi^k / 2. */
void o3_source(int scheme, int m, int n, int l, double h, double d, double alpha,
               const double *phik, const double *phikm1, const double *psik, double *S1,
               double *S2, double *S3) {
    size_t N = (size_t)m * n * l;
    double *tilde = (double *)malloc(N * sizeof(double));
    for (size_t q = 0; q < N; ++q)
        tilde[q] = scheme == 2 ? (3.0 * phik[q] - phikm1[q]) / 2.0 : phik[q];
    for (int k = 0; k < l; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i) {
                size_t q = IX3(i, j, k, m, n);
                S1[q] = phik[q] + d * (psik ? psik[q] : 0.0);
                if (scheme == 1) {
                    S2[q] = 2.0 * lap3(phik, i, j, k, m, n, l, h);
                    S3[q] = 0.0;
                } else {
                    S2[q] = 0.5 * alpha * phik[q] + 2.0 * lap3(tilde, i, j, k, m, n, l, h);
                    S3[q] = 0.5 * lap3(phik, i, j, k, m, n, l, h);
                }
            }
    free(tilde);
}

/* N(u): N1 = phi - c Lap mu, N2 = mu - g(phi) - al phi - Lap kappa,
 * N3 = kappa - e Lap phi. */
void o3_operator(int scheme, int m, int n, int l, double h, double c, double alpha,
                 const double *phik, const double *phi, const double *mu, const double *ka,
                 double *N1, double *N2, double *N3) {
    double al = al3(scheme, alpha), e = e3(scheme);
    for (int k = 0; k < l; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i) {
                size_t q = IX3(i, j, k, m, n);
                double xk = phik ? phik[q] : 0.0;
                N1[q] = phi[q] - c * lap3(mu, i, j, k, m, n, l, h);
                N2[q] = mu[q] - g3(scheme, phi[q], xk) - al * phi[q] - lap3(ka, i, j, k, m, n, l, h);
                N3[q] = ka[q] - e * lap3(phi, i, j, k, m, n, l, h);
            }
}

void o3_residual(int scheme, int m, int n, int l, double h, double c, double alpha,
                 const double *phik, const double *phi, const double *mu, const double *ka,
                 const double *f1, const double *f2, const double *f3, double *r1, double *r2,
                 double *r3) {
    o3_operator(scheme, m, n, l, h, c, alpha, phik, phi, mu, ka, r1, r2, r3);
    size_t N = (size_t)m * n * l;
    for (size_t q = 0; q < N; ++q) {
        r1[q] = f1[q] - r1[q];
        r2[q] = f2[q] - r2[q];
        r3[q] = f3[q] - r3[q];
    }
}

/* sqrt(h^3 sum_c sum r_c^2) */
double o3_norm3(int m, int n, int l, double h, const double *r1, const double *r2,
                const double *r3) {
    size_t N = (size_t)m * n * l;
    double acc = 0.0;
    for (size_t q = 0; q < N; ++q) acc += r1[q] * r1[q] + r2[q] * r2[q] + r3[q] * r3[q];
    return sqrt(h * h * h * acc);
}

/* One cell of the collective smoother: the local 3 x 3 Jacobian of N with
 * respect to the cell's own (phi, mu, kappa) is
 *   [[1, 6c/h^2, 0], [-(al + g'), 1, 6/h^2], [6e/h^2, 0, 1]]
 * (Newton: g' = dg/dphi; Picard: phi^2, resp. chi(phi, phi^k)/2), solved for
 * the correction by Gaussian elimination of the three equations. */
static void relax3(int scheme, int newton, int i, int j, int k, int m, int n, int l, double h,
                   double c, double alpha, const double *phik, double *phi, double *mu,
                   double *ka, const double *f1, const double *f2, const double *f3) {
    size_t q = IX3(i, j, k, m, n);
    double xk = phik ? phik[q] : 0.0, x = phi[q];
    double al = al3(scheme, alpha), e = e3(scheme), ih2 = 1.0 / (h * h);
    double r1 = f1[q] - (x - c * lap3(mu, i, j, k, m, n, l, h));
    double r2 = f2[q] - (mu[q] - g3(scheme, x, xk) - al * x - lap3(ka, i, j, k, m, n, l, h));
    double r3 = f3[q] - (ka[q] - e * lap3(phi, i, j, k, m, n, l, h));
    double dnl = newton ? g3p(scheme, x, xk)
                        : (scheme == 1 ? x * x : 0.5 * (0.5 * (x * x + xk * xk)));
    double A[3][4] = {{1.0, 6.0 * c * ih2, 0.0, r1},
                      {-(al + dnl), 1.0, 6.0 * ih2, r2},
                      {6.0 * e * ih2, 0.0, 1.0, r3}};
    for (int p = 0; p < 3; ++p) {
        int piv = p;
        for (int r = p + 1; r < 3; ++r)
            if (fabs(A[r][p]) > fabs(A[piv][p])) piv = r;
        if (piv != p)
            for (int cc = 0; cc < 4; ++cc) {
                double t = A[p][cc]; A[p][cc] = A[piv][cc]; A[piv][cc] = t;
            }
        for (int r = p + 1; r < 3; ++r) {
            double f = A[r][p] / A[p][p];
            for (int cc = p; cc < 4; ++cc) A[r][cc] -= f * A[p][cc];
        }
    }
    double dk = A[2][3] / A[2][2];
    double dm = (A[1][3] - A[1][2] * dk) / A[1][1];
    double dx = (A[0][3] - A[0][1] * dm - A[0][2] * dk) / A[0][0];
    phi[q] = x + dx;
    mu[q] += dm;
    ka[q] += dk;
}

/* nsweeps red-black passes, red ((i + j + k) even) first. */
void o3_smooth(int scheme, int newton, int nsweeps, int m, int n, int l, double h, double c,
               double alpha, const double *phik, double *phi, double *mu, double *ka,
               const double *f1, const double *f2, const double *f3) {
    for (int s = 0; s < nsweeps; ++s)
        for (int colour = 0; colour < 2; ++colour)
            for (int k = 0; k < l; ++k)
                for (int j = 0; j < n; ++j)
                    for (int i = (j + k + colour) & 1; i < m; i += 2)
                        relax3(scheme, newton, i, j, k, m, n, l, h, c, alpha, phik, phi, mu, ka,
                               f1, f2, f3);
}

/* coarse = average of the 2 x 2 x 2 fine cells under each coarse cell */
void o3_restrict(int m, int n, int l, const double *fine, double *coarse) {
    int mc = m / 2, nc = n / 2, lc = l / 2;
    for (int K = 0; K < lc; ++K)
        for (int J = 0; J < nc; ++J)
            for (int I = 0; I < mc; ++I) {
                double s = 0.0;
                for (int dz = 0; dz < 2; ++dz)
                    for (int dy = 0; dy < 2; ++dy)
                        for (int dx = 0; dx < 2; ++dx)
                            s += fine[IX3(2 * I + dx, 2 * J + dy, 2 * K + dz, m, n)];
                coarse[IX3(I, J, K, mc, nc)] = s / 8.0;
            }
}

/* fine += trilinear interpolation of coarse: per axis the fine cell takes 3/4
 * of its parent's coarse index and 1/4 of the coarse neighbour on its side. */
void o3_prolong_add(int m, int n, int l, const double *coarse, double *fine) {
    int mc = m / 2, nc = n / 2, lc = l / 2;
    for (int k = 0; k < l; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i) {
                int I[2] = {i / 2, wr(i % 2 ? i / 2 + 1 : i / 2 - 1, mc)};
                int J[2] = {j / 2, wr(j % 2 ? j / 2 + 1 : j / 2 - 1, nc)};
                int K[2] = {k / 2, wr(k % 2 ? k / 2 + 1 : k / 2 - 1, lc)};
                const double w[2] = {0.75, 0.25};
                double v = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a)
                            v += w[a] * w[b] * w[c] * coarse[IX3(I[a], J[b], K[c], mc, nc)];
                fine[IX3(i, j, k, m, n)] += v;
            }
}

/* Gaussian elimination with partial pivoting on an nn x nn system. */
static int gauss3(int nn, double *A, double *b) {
    for (int p = 0; p < nn; ++p) {
        int piv = p;
        for (int r = p + 1; r < nn; ++r)
            if (fabs(A[(size_t)r * nn + p]) > fabs(A[(size_t)piv * nn + p])) piv = r;
        if (A[(size_t)piv * nn + p] == 0.0) return -1;
        if (piv != p) {
            for (int cc = 0; cc < nn; ++cc) {
                double t = A[(size_t)p * nn + cc];
                A[(size_t)p * nn + cc] = A[(size_t)piv * nn + cc];
                A[(size_t)piv * nn + cc] = t;
            }
            double t = b[p]; b[p] = b[piv]; b[piv] = t;
        }
        for (int r = p + 1; r < nn; ++r) {
            double f = A[(size_t)r * nn + p] / A[(size_t)p * nn + p];
            if (f == 0.0) continue;
            for (int cc = p; cc < nn; ++cc) A[(size_t)r * nn + cc] -= f * A[(size_t)p * nn + cc];
            b[r] -= f * b[p];
        }
    }
    for (int p = nn - 1; p >= 0; --p) {
        double s = b[p];
        for (int cc = p + 1; cc < nn; ++cc) s -= A[(size_t)p * nn + cc] * b[cc];
        b[p] = s / A[(size_t)p * nn + p];
    }
    return 0;
}

/* Dense Newton on the whole (small) grid: the coarsest level.  Unknowns
 * (phi, mu, kappa) of every cell; the Jacobian of N is assembled column by
 * column from the seven-point stencil.  Returns the iteration count. */
int o3_dense_newton(int scheme, int m, int n, int l, double h, double c, double alpha,
                    const double *phik, double *phi, double *mu, double *ka, const double *f1,
                    const double *f2, const double *f3, int maxit) {
    int N = m * n * l, nn = 3 * N;
    double al = al3(scheme, alpha), e = e3(scheme), ih2 = 1.0 / (h * h);
    double *A = (double *)malloc((size_t)nn * nn * sizeof(double));
    double *b = (double *)malloc((size_t)nn * sizeof(double));
    double *r1 = (double *)malloc((size_t)N * sizeof(double));
    double *r2 = (double *)malloc((size_t)N * sizeof(double));
    double *r3 = (double *)malloc((size_t)N * sizeof(double));
    int it;
    for (it = 1; it <= maxit; ++it) {
        o3_residual(scheme, m, n, l, h, c, alpha, phik, phi, mu, ka, f1, f2, f3, r1, r2, r3);
        memset(A, 0, (size_t)nn * nn * sizeof(double));
        for (int k = 0; k < l; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < m; ++i) {
                    int q = (int)IX3(i, j, k, m, n);
                    int nb[6] = {(int)IX3(wr(i + 1, m), j, k, m, n), (int)IX3(wr(i - 1, m), j, k, m, n),
                                 (int)IX3(i, wr(j + 1, n), k, m, n), (int)IX3(i, wr(j - 1, n), k, m, n),
                                 (int)IX3(i, j, wr(k + 1, l), m, n), (int)IX3(i, j, wr(k - 1, l), m, n)};
                    double xk = phik ? phik[q] : 0.0;
                    size_t r = (size_t)q * nn;            /* row of N1 at q */
                    A[r + q] += 1.0;
                    A[r + N + q] += 6.0 * c * ih2;
                    for (int t = 0; t < 6; ++t) A[r + N + nb[t]] -= c * ih2;
                    r = (size_t)(N + q) * nn;             /* N2 */
                    A[r + N + q] += 1.0;
                    A[r + q] -= al + g3p(scheme, phi[q], xk);
                    A[r + 2 * N + q] += 6.0 * ih2;
                    for (int t = 0; t < 6; ++t) A[r + 2 * N + nb[t]] -= ih2;
                    r = (size_t)(2 * N + q) * nn;         /* N3 */
                    A[r + 2 * N + q] += 1.0;
                    A[r + q] += 6.0 * e * ih2;
                    for (int t = 0; t < 6; ++t) A[r + nb[t]] -= e * ih2;
                    b[q] = r1[q];
                    b[N + q] = r2[q];
                    b[2 * N + q] = r3[q];
                }
        if (gauss3(nn, A, b)) break;
        double dmax = 0.0, xmax = 0.0;
        for (int q = 0; q < N; ++q) {
            phi[q] += b[q];
            mu[q] += b[N + q];
            ka[q] += b[2 * N + q];
            dmax = fmax(dmax, fabs(b[q]));
            xmax = fmax(xmax, fabs(phi[q]));
        }
        if (dmax <= 1e-15 * (1.0 + xmax)) break;
    }
    free(A); free(b); free(r1); free(r2); free(r3);
    return it;
}

typedef struct {
    int m, n, l;
    double h;
    double *u[3], *f[3], *r[3], *v[3], *phik;
} o3_level;

typedef struct {
    int scheme, newton, nu1, nu2, nlev, coarse_sweeps;
    double c, alpha;
    o3_level *L;
} o3_hier;

static void vcycle3(o3_hier *H, int lv) {
    o3_level *A = &H->L[lv];
    if (lv == H->nlev - 1) {
        if (H->coarse_sweeps > 0)
            o3_smooth(H->scheme, H->newton, H->coarse_sweeps, A->m, A->n, A->l, A->h, H->c,
                      H->alpha, A->phik, A->u[0], A->u[1], A->u[2], A->f[0], A->f[1], A->f[2]);
        else
            o3_dense_newton(H->scheme, A->m, A->n, A->l, A->h, H->c, H->alpha, A->phik, A->u[0],
                            A->u[1], A->u[2], A->f[0], A->f[1], A->f[2], 50);
        return;
    }
    o3_level *B = &H->L[lv + 1];
    o3_smooth(H->scheme, H->newton, H->nu1, A->m, A->n, A->l, A->h, H->c, H->alpha, A->phik,
              A->u[0], A->u[1], A->u[2], A->f[0], A->f[1], A->f[2]);
    o3_residual(H->scheme, A->m, A->n, A->l, A->h, H->c, H->alpha, A->phik, A->u[0], A->u[1],
                A->u[2], A->f[0], A->f[1], A->f[2], A->r[0], A->r[1], A->r[2]);
    size_t NB = (size_t)B->m * B->n * B->l;
    for (int f = 0; f < 3; ++f) {
        o3_restrict(A->m, A->n, A->l, A->u[f], B->u[f]);
        memcpy(B->v[f], B->u[f], NB * sizeof(double));
    }
    /* f_H = N_H(restricted u) + restricted residual */
    o3_operator(H->scheme, B->m, B->n, B->l, B->h, H->c, H->alpha, B->phik, B->u[0], B->u[1],
                B->u[2], B->f[0], B->f[1], B->f[2]);
    double *tmp = (double *)malloc(NB * sizeof(double));
    for (int f = 0; f < 3; ++f) {
        o3_restrict(A->m, A->n, A->l, A->r[f], tmp);
        for (size_t q = 0; q < NB; ++q) B->f[f][q] += tmp[q];
    }
    vcycle3(H, lv + 1);
    for (int f = 0; f < 3; ++f) {
        for (size_t q = 0; q < NB; ++q) tmp[q] = B->u[f][q] - B->v[f][q];
        o3_prolong_add(A->m, A->n, A->l, tmp, A->u[f]);
    }
    free(tmp);
    o3_smooth(H->scheme, H->newton, H->nu2, A->m, A->n, A->l, A->h, H->c, H->alpha, A->phik,
              A->u[0], A->u[1], A->u[2], A->f[0], A->f[1], A->f[2]);
}

/* FAS V(nu1, nu2) cycles from the guess in (phi, mu, ka); levels are halved in
 * every axis while the smallest side exceeds `coarsest` and all sides of the
 * next level stay even.  history[0] = ||r|| of the guess, history[c] after
 * cycle c.  Returns the cycles run, or -(cycles + 1) if tol was not reached. */
int o3_fas_solve(int scheme, int newton, int m, int n, int l, double h, double c, double alpha,
                 const double *phik, double *phi, double *mu, double *ka, const double *S1,
                 const double *S2, const double *S3, int nu1, int nu2, int coarsest,
                 int coarse_sweeps, double tol, int max_cycles, double *history) {
    int nlev = 1;
    {
        int a = m, b = n, d = l;
        for (;;) {
            int mn = a < b ? a : b;
            mn = mn < d ? mn : d;
            if (!(mn > coarsest && a % 4 == 0 && b % 4 == 0 && d % 4 == 0)) break;
            a /= 2; b /= 2; d /= 2; ++nlev;
        }
    }
    o3_hier H;
    H.scheme = scheme; H.newton = newton; H.nu1 = nu1; H.nu2 = nu2; H.nlev = nlev;
    H.coarse_sweeps = coarse_sweeps; H.c = c; H.alpha = alpha;
    H.L = (o3_level *)calloc((size_t)nlev, sizeof(o3_level));
    for (int lv = 0; lv < nlev; ++lv) {
        o3_level *A = &H.L[lv];
        A->m = m >> lv; A->n = n >> lv; A->l = l >> lv; A->h = h * (double)(1 << lv);
        size_t N = (size_t)A->m * A->n * A->l;
        for (int f = 0; f < 3; ++f) {
            if (lv == 0) {
                A->u[f] = f == 0 ? phi : (f == 1 ? mu : ka);
                A->f[f] = (double *)(f == 0 ? S1 : (f == 1 ? S2 : S3));
            } else {
                A->u[f] = (double *)calloc(N, sizeof(double));
                A->f[f] = (double *)calloc(N, sizeof(double));
                A->v[f] = (double *)calloc(N, sizeof(double));
            }
            A->r[f] = (double *)calloc(N, sizeof(double));
        }
        if (scheme == 2) {
            if (lv == 0) {
                A->phik = (double *)phik;
            } else {
                A->phik = (double *)calloc(N, sizeof(double));
                o3_restrict(H.L[lv - 1].m, H.L[lv - 1].n, H.L[lv - 1].l, H.L[lv - 1].phik, A->phik);
            }
        } else {
            A->phik = NULL;
        }
    }
    o3_level *F = &H.L[0];
    o3_residual(scheme, m, n, l, h, c, alpha, F->phik, phi, mu, ka, S1, S2, S3, F->r[0], F->r[1],
                F->r[2]);
    double nr = o3_norm3(m, n, l, h, F->r[0], F->r[1], F->r[2]);
    history[0] = nr;
    int cyc = 0;
    while (!(nr <= tol) && cyc < max_cycles) {
        if (nlev == 1 && coarse_sweeps > 0)
            o3_smooth(scheme, newton, coarse_sweeps, m, n, l, h, c, alpha, F->phik, phi, mu, ka,
                      S1, S2, S3);
        else if (nlev == 1)
            o3_dense_newton(scheme, m, n, l, h, c, alpha, F->phik, phi, mu, ka, S1, S2, S3, 50);
        else
            vcycle3(&H, 0);
        ++cyc;
        o3_residual(scheme, m, n, l, h, c, alpha, F->phik, phi, mu, ka, S1, S2, S3, F->r[0],
                    F->r[1], F->r[2]);
        nr = o3_norm3(m, n, l, h, F->r[0], F->r[1], F->r[2]);
        history[cyc] = nr;
        if (!isfinite(nr)) break;
    }
    for (int lv = 0; lv < nlev; ++lv) {
        o3_level *A = &H.L[lv];
        for (int f = 0; f < 3; ++f) {
            if (lv > 0) { free(A->u[f]); free(A->f[f]); free(A->v[f]); }
            free(A->r[f]);
        }
        if (lv > 0 && A->phik) free(A->phik);
    }
    free(H.L);
    return nr <= tol ? cyc : -(cyc + 1);
}

/* kappa = S3 + e Lap phi, then mu = S2 + g(phi) + al phi + Lap kappa, so that
 * N^(3) = S^(3) and N^(2) = S^(2) hold exactly for the guess phi. */
void o3_complete_guess(int scheme, int m, int n, int l, double h, double alpha,
                       const double *phik, const double *phi, double *mu, double *ka,
                       const double *S2, const double *S3) {
    double al = al3(scheme, alpha), e = e3(scheme);
    for (int k = 0; k < l; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i) {
                size_t q = IX3(i, j, k, m, n);
                ka[q] = S3[q] + e * lap3(phi, i, j, k, m, n, l, h);
            }
    for (int k = 0; k < l; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i) {
                size_t q = IX3(i, j, k, m, n);
                double xk = phik ? phik[q] : 0.0;
                mu[q] = S2[q] + g3(scheme, phi[q], xk) + al * phi[q] + lap3(ka, i, j, k, m, n, l, h);
            }
}

/* ||grad_h f||^2 = h^3 sum over east, north, top faces of (difference / h)^2. */
double o3_grad_sq(int m, int n, int l, double h, const double *f) {
    double s = 0.0;
    for (int k = 0; k < l; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i) {
                double x = f[IX3(i, j, k, m, n)];
                double dx = f[IX3(wr(i + 1, m), j, k, m, n)] - x;
                double dy = f[IX3(i, wr(j + 1, n), k, m, n)] - x;
                double dz = f[IX3(i, j, wr(k + 1, l), m, n)] - x;
                s += dx * dx + dy * dy + dz * dz;
            }
    return h * s;
}

/* F = 1/4 ||phi||_4^4 + alpha/2 ||phi||^2 - ||grad_h phi||^2 + 1/2 ||Lap_h phi||^2
 * with ||f||_p^p = h^3 sum |f|^p (eq. discrete_energy_PFC in three dimensions). */
double o3_energy_F(int m, int n, int l, double h, double eps, const double *phi) {
    double alpha = 1.0 - eps, h3 = h * h * h;
    double s4 = 0.0, s2 = 0.0, sl = 0.0;
    for (int k = 0; k < l; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i) {
                double x = phi[IX3(i, j, k, m, n)];
                double L = lap3(phi, i, j, k, m, n, l, h);
                s4 += x * x * x * x;
                s2 += x * x;
                sl += L * L;
            }
    return 0.25 * h3 * s4 + 0.5 * alpha * h3 * s2 - o3_grad_sq(m, n, l, h, phi) + 0.5 * h3 * sl;
}

/* -Lap_h w = b - mean(b), mean(w) = 0, by conjugate gradients to
 * ||r|| <= rtol ||b - mean(b)||.  Returns the iterations (-1: maxit reached). */
int o3_poisson_cg(int m, int n, int l, double h, const double *b, double *w, double rtol,
                  int maxit) {
    size_t N = (size_t)m * n * l;
    double *r = (double *)malloc(N * sizeof(double));
    double *p = (double *)malloc(N * sizeof(double));
    double *Ap = (double *)malloc(N * sizeof(double));
    double mean = 0.0;
    for (size_t q = 0; q < N; ++q) mean += b[q];
    mean /= (double)N;
    double bn = 0.0;
    for (size_t q = 0; q < N; ++q) {
        w[q] = 0.0;
        r[q] = b[q] - mean;
        p[q] = r[q];
        bn += r[q] * r[q];
    }
    double rr = bn;
    int it = 0, ret = bn == 0.0 ? 0 : -1;
    for (it = 1; ret < 0 && it <= maxit; ++it) {
        for (int k = 0; k < l; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < m; ++i)
                    Ap[IX3(i, j, k, m, n)] = -lap3(p, i, j, k, m, n, l, h);
        double pAp = 0.0;
        for (size_t q = 0; q < N; ++q) pAp += p[q] * Ap[q];
        double a = rr / pAp, rr2 = 0.0;
        for (size_t q = 0; q < N; ++q) {
            w[q] += a * p[q];
            r[q] -= a * Ap[q];
            rr2 += r[q] * r[q];
        }
        if (sqrt(rr2) <= rtol * sqrt(bn)) { ret = it; break; }
        double beta = rr2 / rr;
        rr = rr2;
        for (size_t q = 0; q < N; ++q) p[q] = r[q] + beta * p[q];
    }
    double mw = 0.0;
    for (size_t q = 0; q < N; ++q) mw += w[q];
    mw /= (double)N;
    for (size_t q = 0; q < N; ++q) w[q] -= mw;
    free(r); free(p); free(Ap);
    return ret;
}

/* out[0] = F(phi^{k+1}), out[1] = F + ||psi||_{-1}^2 / (2M) with
 * ||psi||_{-1}^2 = h^3 (psi - mean psi, w), -Lap_h w = psi - mean psi,
 * out[2] = out[1] + ||grad_h(phi^{k+1} - phi^k)||^2 / 2, out[3] = h^3 sum phi. */
void o3_energies(int m, int n, int l, double h, double eps, double M, const double *phinew,
                 const double *phik, const double *psinew, double *out) {
    size_t N = (size_t)m * n * l;
    double h3 = h * h * h;
    double F = o3_energy_F(m, n, l, h, eps, phinew);
    double *w = (double *)malloc(N * sizeof(double));
    double *d = (double *)malloc(N * sizeof(double));
    o3_poisson_cg(m, n, l, h, psinew, w, 1e-14, 100000);
    double mean = 0.0, mass = 0.0;
    for (size_t q = 0; q < N; ++q) mean += psinew[q];
    mean /= (double)N;
    double acc = 0.0;
    for (size_t q = 0; q < N; ++q) {
        acc += (psinew[q] - mean) * w[q];
        d[q] = phinew[q] - phik[q];
        mass += phinew[q];
    }
    out[0] = F;
    out[1] = F + h3 * acc / (2.0 * M);
    out[2] = out[1] + 0.5 * o3_grad_sq(m, n, l, h, d);
    out[3] = h3 * mass;
    free(w); free(d);
}

/* One time step in three dimensions (Sec. 3.1 / 3.2 with App. B): source,
 * guess (phi^k, or 2 phi^k - phi^{k-1} for guess = 1) completed in mu and
 * kappa, FAS V-cycles, psi update (eq. discrete_1_b / discrete_2_b), energies
 * (if `energies` is not NULL).  Returns the cycles (negative: tol not met). */
int o3_step(int scheme, int newton, int m, int n, int l, double h, double s, double M,
            double beta, double eps, const double *phik, const double *phikm1,
            const double *psik, int guess, int nu1, int nu2, int coarsest, int coarse_sweeps,
            double tol, int max_cycles, double *phinew, double *mu, double *ka,
            double *psinew, double *history, double *energies) {
    size_t N = (size_t)m * n * l;
    double q = scheme == 1 ? 1.0 : 2.0;
    double c = s * M / (beta + q / s), d = q / (beta + q / s), alpha = 1.0 - eps;
    double *S1 = (double *)malloc(N * sizeof(double));
    double *S2 = (double *)malloc(N * sizeof(double));
    double *S3 = (double *)malloc(N * sizeof(double));
    o3_source(scheme, m, n, l, h, d, alpha, phik, phikm1, psik, S1, S2, S3);
    for (size_t p = 0; p < N; ++p) phinew[p] = guess == 1 ? 2.0 * phik[p] - phikm1[p] : phik[p];
    const double *pk = scheme == 2 ? phik : NULL;
    o3_complete_guess(scheme, m, n, l, h, alpha, pk, phinew, mu, ka, S2, S3);
    int cyc = o3_fas_solve(scheme, newton, m, n, l, h, c, alpha, pk, phinew, mu, ka, S1, S2, S3,
                           nu1, nu2, coarsest, coarse_sweeps, tol, max_cycles, history);
    for (size_t p = 0; p < N; ++p)
        psinew[p] = scheme == 1 ? (phinew[p] - phik[p]) / s
                                : (2.0 / s) * (phinew[p] - phik[p]) - (psik ? psik[p] : 0.0);
    if (energies) o3_energies(m, n, l, h, eps, M, phinew, phik, psinew, energies);
    free(S1); free(S2); free(S3);
    return cyc;
}
