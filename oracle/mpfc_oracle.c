/*
 * mpfc_oracle.c -- plain, slow, FP64 CPU oracle for one implicit time step of
 * the two convex-splitting schemes for the modified phase field crystal (MPFC)
 * equation on a periodic cell-centred grid (Baskaran, Zhou, Hu, Wang, Wise,
 * Lowengrub, "Energy stable and efficient finite-difference nonlinear
 * multigrid schemes for the modified phase field crystal equation").
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists to check the GPU library.  Only
 * the test suite, the package smoke check and the CPU-baseline leg of the
 * benchmark may load it.  The product path never calls it, and it shares no
 * code, header, table or helper with the HIP sources.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fused
 * multiply-add, so every sum is evaluated as written).
 *
 * Notation follows the paper: grid m x n, spacing h, time step s, mobility M,
 * damping beta, alpha = 1 - eps.  Cells (i, j), 0 <= i < m, 0 <= j < n, are
 * stored row-major with i (x) fastest: index j*m + i.  Ghost values (App. A)
 * are realised by index mapping, per axis: periodic boundary conditions by
 * wrap-around, homogeneous Neumann conditions by repeating the boundary cell
 * (orc_set_bc selects the conditions; periodic in both directions unless set).
 *
 * Unknown u = (phi, mu, kappa), three m x n fields (App. B.1 / B.2).
 *
 * Readings of points the paper leaves open (each one is listed with its reason
 * in the design notes of the repository):
 *  - the local 3x3 system of the smoother is solved in correction form:
 *    J_loc * delta = (S - N(u))_{ij}, then u_{ij} += delta, where J_loc is the
 *    derivative of N at cell (i,j) with respect to that cell's own unknowns.
 *    For Picard linearisation this is algebraically the smoother printed in
 *    App. B.1; for scheme 2 it also avoids the misprinted factor 4 in the
 *    first smoother equation of App. B.2 (the fixed point must be N = S);
 *  - red-black ordering, red = (i + j) even, red first (App. B.1 says the
 *    codes use red-black ordering);
 *  - standard FAS V-cycle: restriction of u and of the residual by the
 *    average of the 2x2 fine cells under a coarse cell, bilinear
 *    (9/16, 3/16, 3/16, 1/16) prolongation, coarsest grid solved by dense
 *    Newton iteration with Gaussian elimination (partial pivoting);
 *  - the residual norm is sqrt(h^2 * sum over the three components of r^2),
 *    the h-weighted discrete l2 norm of App. A applied to all of r;
 *  - scheme-2 coarse operators use phi^k restricted by the same 2x2 average;
 *  - pinning (Sec. 4.6, scheme 2): mu is replaced by
 *    mu~ = mu + 2 (phi^{k+1/2} - phi_hat) W with phi^{k+1/2} = (phi^{k+1} + phi^k)/2
 *    and the weight W; taking mu~ as the unknown gives N^(2) an extra -W phi
 *    and S^(2) an extra W (phi^k - 2 phi_hat); coarse levels use W restricted
 *    by the 2x2 average, and the reported energy F gains h^2 sum W (phi - phi_hat)^2
 *    (the discrete form of the added integral);
 *  - grids whose sides are not powers of two (Sec. 4.6 uses 512 x 400) coarsen
 *    while both sides of the next level stay even; the coarsest level may
 *    then be too large for the dense Newton solve and is instead relaxed by
 *    a fixed number of the same red-black sweeps;
 *  - on a homogeneous Neumann boundary the ghost cell (a copy of the boundary
 *    cell) enters the smoother's neighbour sums with the value it has before
 *    the cell is updated (ghosts refreshed before every half-sweep), and the
 *    smoother's local 3x3 matrix stays the interior one; the residual, the
 *    transfers (the coarse ghost repeats the boundary coarse cell) and the
 *    coarsest-grid Newton matrix use the ghost rule exactly;
 *  - optional under-relaxation of the smoother (orc_set_omega; default 1, the
 *    update of App. B unchanged): each cell moves by omega times its local
 *    correction.  A local Fourier analysis of the linearised App. B smoother
 *    shows it amplifies a band of error modes (spectral radius of one
 *    red-black pass up to about 1.3) whenever c/h^4 lies in an intermediate
 *    range; V-cycles then diverge for some time steps (first-order scheme,
 *    h = 0.5: s from about 0.15 to 0.3), and omega near 0.8 restores a
 *    contraction of about 0.2 per V(2,2) cycle there.  The fixed point (the
 *    discrete solution) does not depend on omega.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IX(i, j, m) ((size_t)(j) * (size_t)(m) + (size_t)(i))

/* Boundary conditions of the two axes (App. A): 0 = periodic, 1 = homogeneous
 * Neumann.  Process-wide setting read by every routine below. */
static int g_neumann_x = 0, g_neumann_y = 0;

void orc_set_bc(int neumann_x, int neumann_y) {
    g_neumann_x = neumann_x != 0;
    g_neumann_y = neumann_y != 0;
}

/* Cell index of the ghost or interior cell i in [-1, m] along one axis, for
 * 0-based indices.  Periodic (eqs. per-bcs): ghost 0 is cell m and ghost m+1
 * is cell 1 in the paper's 1-based numbering.  Homogeneous Neumann (eqs.
 * h-n-bcs): ghost 0 repeats cell 1 and ghost m+1 repeats cell m. */
static int ghost_index(int i, int m, int neumann) {
    if (i < 0) return neumann ? 0 : i + m;
    if (i >= m) return neumann ? m - 1 : i - m;
    return i;
}
static int wrapx(int i, int m) { return ghost_index(i, m, g_neumann_x); }
static int wrapy(int j, int n) { return ghost_index(j, n, g_neumann_y); }

/* ------------------------------------------------------------------------ */
/* Discrete operators (App. A).                                             */
/* ------------------------------------------------------------------------ */

/* Standard five-point Laplacian, Delta_h f = (f_E + f_W + f_N + f_S - 4 f)/h^2. */
static double lap_at(const double *f, int i, int j, int m, int n, double h) {
    double fe = f[IX(wrapx(i + 1, m), j, m)];
    double fw = f[IX(wrapx(i - 1, m), j, m)];
    double fn = f[IX(i, wrapy(j + 1, n), m)];
    double fs = f[IX(i, wrapy(j - 1, n), m)];
    double fc = f[IX(i, j, m)];
    return (fe + fw + fn + fs - 4.0 * fc) / (h * h);
}

void orc_laplacian(int m, int n, double h, const double *f, double *out) {
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i)
            out[IX(i, j, m)] = lap_at(f, i, j, m, n, h);
}

/* ------------------------------------------------------------------------ */
/* Scheme coefficients (Sec. 3.1 eq. discrete_1_a, Sec. 3.2 eq. discrete_2_a) */
/* ------------------------------------------------------------------------ */

typedef struct {
    int scheme;      /* 1: first-order convex splitting; 2: second order */
    double h, s, M, beta, eps;
} orc_model;

/* c = s M / (beta + 1/s) (scheme 1) or s M / (beta + 2/s) (scheme 2);
 * d = 1 / (beta + 1/s) or 2 / (beta + 2/s), the weight of psi^k. */
void orc_coefficients(const orc_model *p, double *c, double *d) {
    if (p->scheme == 1) {
        *c = p->s * p->M / (p->beta + 1.0 / p->s);
        *d = 1.0 / (p->beta + 1.0 / p->s);
    } else {
        *c = p->s * p->M / (p->beta + 2.0 / p->s);
        *d = 2.0 / (p->beta + 2.0 / p->s);
    }
}

/* Nonlinear term of N^(2) and its derivative.
 * Scheme 1 (App. B.1): phi^3.
 * Scheme 2 (App. B.2): (1/2) chi(phi, phi^k) (phi + phi^k) with
 * chi(a, b) = (a^2 + b^2)/2 (Sec. 3.2). */
static double gnl(int scheme, double x, double xk) {
    if (scheme == 1) return x * x * x;
    return 0.5 * (0.5 * (x * x + xk * xk)) * (x + xk);
}
static double gnl_prime(int scheme, double x, double xk) {
    if (scheme == 1) return 3.0 * x * x;
    /* d/dx of (x^2 + xk^2)(x + xk)/4 = (2x(x + xk) + x^2 + xk^2)/4 */
    return (2.0 * x * (x + xk) + x * x + xk * xk) / 4.0;
}
/* Linear coefficient of phi in N^(2): alpha (scheme 1), alpha/2 (scheme 2). */
static double alin(int scheme, double alpha) { return scheme == 1 ? alpha : 0.5 * alpha; }
/* Coefficient of Delta_h phi in N^(3): 1 (scheme 1), 1/2 (scheme 2). */
static double ecoef(int scheme) { return scheme == 1 ? 1.0 : 0.5; }

/* Source S (App. B.1 and B.2). phikm1 and psik may be NULL where unused. */
void orc_source(const orc_model *p, int m, int n, const double *phik, const double *phikm1,
                const double *psik, double *S1, double *S2, double *S3, const double *pin,
                const double *phihat) {
    double c, d;
    orc_coefficients(p, &c, &d);
    double alpha = 1.0 - p->eps;
    double h = p->h;
    size_t N = (size_t)m * n;
    double *tilde = (double *)malloc(N * sizeof(double));
    for (size_t q = 0; q < N; ++q) {
        /* second-order extrapolation phi~^{k+1/2} = (3 phi^k - phi^{k-1})/2 (Sec. 3.2) */
        tilde[q] = (p->scheme == 2) ? (3.0 * phik[q] - phikm1[q]) / 2.0 : phik[q];
    }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            size_t q = IX(i, j, m);
            double ps = psik ? psik[q] : 0.0;
            S1[q] = phik[q] + d * ps;
            if (p->scheme == 1) {
                S2[q] = 2.0 * lap_at(phik, i, j, m, n, h);
                S3[q] = 0.0;
            } else {
                S2[q] = 0.5 * alpha * phik[q] + 2.0 * lap_at(tilde, i, j, m, n, h);
                if (pin) S2[q] += pin[q] * (phik[q] - 2.0 * phihat[q]);
                S3[q] = 0.5 * lap_at(phik, i, j, m, n, h);
            }
        }
    free(tilde);
}

/* N(u) on an m x n grid with spacing h (App. B.1 and B.2).  phik is used by
 * scheme 2 only (may be NULL for scheme 1); pin is the pinning weight on this
 * grid (NULL: none). */
void orc_operator(int scheme, int m, int n, double h, double c, double alpha,
                  const double *phik, const double *phi, const double *mu, const double *ka,
                  double *N1, double *N2, double *N3, const double *pin) {
    double al = alin(scheme, alpha), e = ecoef(scheme);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            size_t q = IX(i, j, m);
            double xk = phik ? phik[q] : 0.0;
            N1[q] = phi[q] - c * lap_at(mu, i, j, m, n, h);
            double alq = al + (pin ? pin[q] : 0.0);
            N2[q] = mu[q] - gnl(scheme, phi[q], xk) - alq * phi[q] - lap_at(ka, i, j, m, n, h);
            N3[q] = ka[q] - e * lap_at(phi, i, j, m, n, h);
        }
}

/* r = f - N(u) */
void orc_residual(int scheme, int m, int n, double h, double c, double alpha,
                  const double *phik, const double *phi, const double *mu, const double *ka,
                  const double *f1, const double *f2, const double *f3,
                  double *r1, double *r2, double *r3, const double *pin) {
    orc_operator(scheme, m, n, h, c, alpha, phik, phi, mu, ka, r1, r2, r3, pin);
    size_t N = (size_t)m * n;
    for (size_t q = 0; q < N; ++q) {
        r1[q] = f1[q] - r1[q];
        r2[q] = f2[q] - r2[q];
        r3[q] = f3[q] - r3[q];
    }
}

/* sqrt(h^2 * sum_c sum_ij r_c^2) */
double orc_norm3(int m, int n, double h, const double *r1, const double *r2, const double *r3) {
    size_t N = (size_t)m * n;
    double acc = 0.0;
    for (size_t q = 0; q < N; ++q) acc += r1[q] * r1[q] + r2[q] * r2[q] + r3[q] * r3[q];
    return sqrt(h * h * acc);
}

/* ------------------------------------------------------------------------ */
/* Nonlinear red-black Gauss-Seidel smoothing (App. B.1, B.2).              */
/* ------------------------------------------------------------------------ */

/* 3x3 determinant of rows (a0,a1,a2),(b0,b1,b2),(c0,c1,c2). */
static double det3(double a0, double a1, double a2, double b0, double b1, double b2,
                   double c0, double c1, double c2) {
    return a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0);
}

/* Update one cell: local linearisation of the cubic term (Newton or Picard,
 * App. B.1), then the 3x3 system in the cell's own unknowns solved by
 * Cramer's rule (App. B.1, B.2).  The right-hand side is the current residual
 * at the cell (correction form). */
/* Relaxation factor of the cell update (orc_set_omega): the smoother moves
 * each cell by omega times the solution of its local 3x3 system.  omega = 1
 * is the collective Gauss-Seidel update of App. B; 0 < omega < 1
 * under-relaxes it (not in the paper: a reading adopted because App. B's
 * update amplifies a band of error modes whenever c/h^4 lies in an
 * intermediate range, where V-cycles then diverge; see the file header). */
static double g_omega = 1.0;

void orc_set_omega(double omega) { g_omega = omega; }

static void relax_cell(int scheme, int newton, int i, int j, int m, int n, double h, double c,
                       double alpha, const double *phik, double *phi, double *mu, double *ka,
                       const double *f1, const double *f2, const double *f3, const double *pin) {
    size_t q = IX(i, j, m);
    double xk = phik ? phik[q] : 0.0;
    double x = phi[q];
    double al = alin(scheme, alpha) + (pin ? pin[q] : 0.0), e = ecoef(scheme);
    double r1 = f1[q] - (x - c * lap_at(mu, i, j, m, n, h));
    double r2 = f2[q] - (mu[q] - gnl(scheme, x, xk) - al * x - lap_at(ka, i, j, m, n, h));
    double r3 = f3[q] - (ka[q] - e * lap_at(phi, i, j, m, n, h));
    /* derivative of N at (i,j) w.r.t. (phi_ij, mu_ij, kappa_ij) */
    double dnl;
    if (newton) {
        dnl = gnl_prime(scheme, x, xk);
    } else if (scheme == 1) {
        dnl = x * x; /* Picard: phi^3 ~ phi_l^2 phi */
    } else {
        dnl = 0.5 * (0.5 * (x * x + xk * xk)); /* Picard: chi(phi_l, phi^k)/2 */
    }
    double a11 = 1.0, a12 = 4.0 * c / (h * h), a13 = 0.0;
    double a21 = -(al + dnl), a22 = 1.0, a23 = 4.0 / (h * h);
    double a31 = 4.0 * e / (h * h), a32 = 0.0, a33 = 1.0;
    double D = det3(a11, a12, a13, a21, a22, a23, a31, a32, a33);
    double dx = det3(r1, a12, a13, r2, a22, a23, r3, a32, a33) / D;
    double dm = det3(a11, r1, a13, a21, r2, a23, a31, r3, a33) / D;
    double dk = det3(a11, a12, r1, a21, a22, r2, a31, a32, r3) / D;
    phi[q] = x + g_omega * dx;
    mu[q] += g_omega * dm;
    ka[q] += g_omega * dk;
}

/* One half-sweep over the cells of one colour (colour = (i + j) mod 2,
 * 0 = red).  Cells of one colour only couple to the other colour. */
void orc_smooth_color(int scheme, int newton, int color, int m, int n, double h, double c,
                      double alpha, const double *phik, double *phi, double *mu, double *ka,
                      const double *f1, const double *f2, const double *f3, const double *pin) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j)
        for (int i = (j + color) & 1; i < m; i += 2)
            relax_cell(scheme, newton, i, j, m, n, h, c, alpha, phik, phi, mu, ka, f1, f2, f3, pin);
}

/* nsweeps full red-black passes ("ell_max" smoothing iterations, App. B.1). */
void orc_smooth(int scheme, int newton, int nsweeps, int m, int n, double h, double c,
                double alpha, const double *phik, double *phi, double *mu, double *ka,
                const double *f1, const double *f2, const double *f3, const double *pin) {
    for (int l = 0; l < nsweeps; ++l) {
        orc_smooth_color(scheme, newton, 0, m, n, h, c, alpha, phik, phi, mu, ka, f1, f2, f3, pin);
        orc_smooth_color(scheme, newton, 1, m, n, h, c, alpha, phik, phi, mu, ka, f1, f2, f3, pin);
    }
}

/* Lexicographic nonlinear Gauss-Seidel pass, the ordering printed in App. B
 * (used only to check that the ordering does not change the fixed point). */
void orc_smooth_lex(int scheme, int newton, int nsweeps, int m, int n, double h, double c,
                    double alpha, const double *phik, double *phi, double *mu, double *ka,
                    const double *f1, const double *f2, const double *f3, const double *pin) {
    for (int l = 0; l < nsweeps; ++l)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i)
                relax_cell(scheme, newton, i, j, m, n, h, c, alpha, phik, phi, mu, ka, f1, f2, f3, pin);
}

/* ------------------------------------------------------------------------ */
/* Grid transfers of the FAS V-cycle.                                       */
/* ------------------------------------------------------------------------ */

/* coarse (m/2 x n/2) = average of the 2x2 fine cells under each coarse cell */
void orc_restrict(int m, int n, const double *fine, double *coarse) {
    int mc = m / 2, nc = n / 2;
    for (int J = 0; J < nc; ++J)
        for (int I = 0; I < mc; ++I) {
            double s = fine[IX(2 * I, 2 * J, m)] + fine[IX(2 * I + 1, 2 * J, m)] +
                       fine[IX(2 * I, 2 * J + 1, m)] + fine[IX(2 * I + 1, 2 * J + 1, m)];
            coarse[IX(I, J, mc)] = 0.25 * s;
        }
}

/* fine (m x n) += bilinear interpolation of the coarse field (m/2 x n/2).
 * A fine cell lies in one quadrant of its coarse parent; its value is
 * 9/16 of the parent, 3/16 of each of the two coarse neighbours on the
 * quadrant's sides and 1/16 of the diagonal coarse neighbour. */
void orc_prolong_add(int m, int n, const double *coarse, double *fine) {
    int mc = m / 2, nc = n / 2;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            int I = i / 2, J = j / 2;
            int Is = wrapx((i % 2 == 0) ? I - 1 : I + 1, mc);
            int Js = wrapy((j % 2 == 0) ? J - 1 : J + 1, nc);
            double v = 9.0 * coarse[IX(I, J, mc)] + 3.0 * coarse[IX(Is, J, mc)] +
                       3.0 * coarse[IX(I, Js, mc)] + 1.0 * coarse[IX(Is, Js, mc)];
            fine[IX(i, j, m)] += v / 16.0;
        }
}

/* ------------------------------------------------------------------------ */
/* Dense Newton solve of N(u) = f on a (small) grid: the coarsest level.    */
/* ------------------------------------------------------------------------ */

/* Solve A x = b (A is nn x nn, row-major, overwritten) by Gaussian
 * elimination with partial pivoting.  Returns 0, or -1 if singular. */
static int gauss_solve(int nn, double *A, double *b) {
    for (int k = 0; k < nn; ++k) {
        int piv = k;
        double best = fabs(A[(size_t)k * nn + k]);
        for (int r = k + 1; r < nn; ++r) {
            double v = fabs(A[(size_t)r * nn + k]);
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) return -1;
        if (piv != k) {
            for (int cc = 0; cc < nn; ++cc) {
                double t = A[(size_t)k * nn + cc];
                A[(size_t)k * nn + cc] = A[(size_t)piv * nn + cc];
                A[(size_t)piv * nn + cc] = t;
            }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int r = k + 1; r < nn; ++r) {
            double fct = A[(size_t)r * nn + k] / A[(size_t)k * nn + k];
            if (fct == 0.0) continue;
            for (int cc = k; cc < nn; ++cc) A[(size_t)r * nn + cc] -= fct * A[(size_t)k * nn + cc];
            b[r] -= fct * b[k];
        }
    }
    for (int k = nn - 1; k >= 0; --k) {
        double s = b[k];
        for (int cc = k + 1; cc < nn; ++cc) s -= A[(size_t)k * nn + cc] * b[cc];
        b[k] = s / A[(size_t)k * nn + k];
    }
    return 0;
}

/* Newton iteration on the full 3*m*n system N(u) = f with the exact Jacobian,
 * unknown ordering (phi over cells, then mu, then kappa).  Iterates until the
 * max-norm of the Newton step is below 1e-15 * (1 + max|u|), at most maxit
 * times.  Returns the number of iterations, or -1 on a singular Jacobian. */
int orc_dense_newton(int scheme, int m, int n, double h, double c, double alpha,
                     const double *phik, double *phi, double *mu, double *ka,
                     const double *f1, const double *f2, const double *f3, int maxit,
                     const double *pin) {
    int nc = m * n, nn = 3 * nc;
    double *A = (double *)malloc((size_t)nn * nn * sizeof(double));
    double *b = (double *)malloc((size_t)nn * sizeof(double));
    double *r1 = (double *)malloc((size_t)nc * sizeof(double));
    double *r2 = (double *)malloc((size_t)nc * sizeof(double));
    double *r3 = (double *)malloc((size_t)nc * sizeof(double));
    double al = alin(scheme, alpha), e = ecoef(scheme), ih2 = 1.0 / (h * h);
    int it, ret = -1;
    for (it = 1; it <= maxit; ++it) {
        orc_residual(scheme, m, n, h, c, alpha, phik, phi, mu, ka, f1, f2, f3, r1, r2, r3, pin);
        memset(A, 0, (size_t)nn * nn * sizeof(double));
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i) {
                int q = (int)IX(i, j, m);
                int nb[4] = {(int)IX(wrapx(i + 1, m), j, m), (int)IX(wrapx(i - 1, m), j, m),
                             (int)IX(i, wrapy(j + 1, n), m), (int)IX(i, wrapy(j - 1, n), m)};
                double xk = phik ? phik[q] : 0.0;
                /* row of N^(1): phi - c Lap(mu) */
                A[(size_t)q * nn + q] += 1.0;
                A[(size_t)q * nn + nc + q] += 4.0 * c * ih2;
                for (int t = 0; t < 4; ++t) A[(size_t)q * nn + nc + nb[t]] -= c * ih2;
                /* row of N^(2): mu - g(phi) - al phi - Lap(kappa) */
                size_t r = (size_t)(nc + q) * nn;
                A[r + q] -= al + (pin ? pin[q] : 0.0) + gnl_prime(scheme, phi[q], xk);
                A[r + nc + q] += 1.0;
                A[r + 2 * nc + q] += 4.0 * ih2;
                for (int t = 0; t < 4; ++t) A[r + 2 * nc + nb[t]] -= ih2;
                /* row of N^(3): kappa - e Lap(phi) */
                r = (size_t)(2 * nc + q) * nn;
                A[r + 2 * nc + q] += 1.0;
                A[r + q] += 4.0 * e * ih2;
                for (int t = 0; t < 4; ++t) A[r + nb[t]] -= e * ih2;
                b[q] = r1[q];
                b[nc + q] = r2[q];
                b[2 * nc + q] = r3[q];
            }
        if (gauss_solve(nn, A, b) != 0) { ret = -1; goto done; }
        double step = 0.0, size = 0.0;
        for (int q = 0; q < nc; ++q) {
            phi[q] += b[q];
            mu[q] += b[nc + q];
            ka[q] += b[2 * nc + q];
            double s3 = fmax(fabs(b[q]), fmax(fabs(b[nc + q]), fabs(b[2 * nc + q])));
            double u3 = fmax(fabs(phi[q]), fmax(fabs(mu[q]), fabs(ka[q])));
            step = fmax(step, s3);
            size = fmax(size, u3);
        }
        if (step <= 1e-15 * (1.0 + size)) break;
    }
    ret = it > maxit ? maxit : it;
done:
    free(A); free(b); free(r1); free(r2); free(r3);
    return ret;
}

/* ------------------------------------------------------------------------ */
/* FAS V-cycle (standard full approximation scheme; App. B refers the other */
/* components to the multigrid literature).                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    int m, n;
    double h;
    double *u[3], *f[3], *r[3], *v[3], *phik, *pin;
} orc_level;

typedef struct {
    int scheme, newton, nu1, nu2, nlev;
    int coarse_sweeps;  /* 0: dense Newton on the coarsest grid; K > 0: K red-black sweeps */
    double c, alpha;
    orc_level *L;
} orc_hier;

static void vcycle(orc_hier *H, int l) {
    orc_level *A = &H->L[l];
    if (l == H->nlev - 1) {
        if (H->coarse_sweeps > 0)
            orc_smooth(H->scheme, H->newton, H->coarse_sweeps, A->m, A->n, A->h, H->c, H->alpha,
                       A->phik, A->u[0], A->u[1], A->u[2], A->f[0], A->f[1], A->f[2], A->pin);
        else
            orc_dense_newton(H->scheme, A->m, A->n, A->h, H->c, H->alpha, A->phik, A->u[0],
                             A->u[1], A->u[2], A->f[0], A->f[1], A->f[2], 50, A->pin);
        return;
    }
    orc_level *B = &H->L[l + 1];
    orc_smooth(H->scheme, H->newton, H->nu1, A->m, A->n, A->h, H->c, H->alpha, A->phik, A->u[0],
               A->u[1], A->u[2], A->f[0], A->f[1], A->f[2], A->pin);
    orc_residual(H->scheme, A->m, A->n, A->h, H->c, H->alpha, A->phik, A->u[0], A->u[1], A->u[2],
                 A->f[0], A->f[1], A->f[2], A->r[0], A->r[1], A->r[2], A->pin);
    size_t NB = (size_t)B->m * B->n;
    for (int k = 0; k < 3; ++k) {
        orc_restrict(A->m, A->n, A->u[k], B->u[k]);
        memcpy(B->v[k], B->u[k], NB * sizeof(double));
    }
    /* f_H = N_H(restricted u) + restricted residual */
    orc_operator(H->scheme, B->m, B->n, B->h, H->c, H->alpha, B->phik, B->u[0], B->u[1], B->u[2],
                 B->f[0], B->f[1], B->f[2], B->pin);
    double *tmp = (double *)malloc(NB * sizeof(double));
    for (int k = 0; k < 3; ++k) {
        orc_restrict(A->m, A->n, A->r[k], tmp);
        for (size_t q = 0; q < NB; ++q) B->f[k][q] += tmp[q];
    }
    vcycle(H, l + 1);
    for (int k = 0; k < 3; ++k) {
        for (size_t q = 0; q < NB; ++q) tmp[q] = B->u[k][q] - B->v[k][q];
        orc_prolong_add(A->m, A->n, tmp, A->u[k]);
    }
    free(tmp);
    orc_smooth(H->scheme, H->newton, H->nu2, A->m, A->n, A->h, H->c, H->alpha, A->phik, A->u[0],
               A->u[1], A->u[2], A->f[0], A->f[1], A->f[2], A->pin);
}

/* Solve N(u) = S by FAS V(nu1, nu2) cycles on levels m x n, m/2 x n/2, ...
 * A level is coarsened while its smaller side exceeds `coarsest` and both
 * sides of the next level are even (the red-black colouring of a periodic
 * axis needs an even number of cells), so 512 x 400 stops at 64 x 50.
 * The coarsest grid is solved by dense Newton (coarse_sweeps = 0) or
 * approximately by coarse_sweeps red-black sweeps, for grids whose coarsest
 * level is too large for a dense solve.
 * u holds the initial guess on entry and the last iterate on exit.
 * history[0] = ||r|| of the guess, history[k] = ||r|| after cycle k
 * (history has room for max_cycles + 1 entries).  Returns the number of
 * cycles run, or -(cycles + 1) if the tolerance was not reached. */
int orc_fas_solve(int scheme, int newton, int m, int n, double h, double c, double alpha,
                  const double *phik, double *phi, double *mu, double *ka, const double *S1,
                  const double *S2, const double *S3, int nu1, int nu2, int coarsest,
                  int coarse_sweeps, double tol, int max_cycles, double *history,
                  const double *pin) {
    int nlev = 1;
    {
        int mm = m, nn = n;
        while ((mm < nn ? mm : nn) > coarsest && mm % 4 == 0 && nn % 4 == 0) {
            mm /= 2; nn /= 2; ++nlev;
        }
    }
    orc_hier H;
    H.scheme = scheme; H.newton = newton; H.nu1 = nu1; H.nu2 = nu2; H.nlev = nlev;
    H.coarse_sweeps = coarse_sweeps;
    H.c = c; H.alpha = alpha;
    H.L = (orc_level *)calloc((size_t)nlev, sizeof(orc_level));
    for (int l = 0; l < nlev; ++l) {
        orc_level *A = &H.L[l];
        A->m = m >> l; A->n = n >> l; A->h = h * (double)(1 << l);
        size_t N = (size_t)A->m * A->n;
        for (int k = 0; k < 3; ++k) {
            if (l == 0) {
                A->u[k] = (k == 0 ? phi : (k == 1 ? mu : ka));
                A->f[k] = (double *)(k == 0 ? S1 : (k == 1 ? S2 : S3));
            } else {
                A->u[k] = (double *)calloc(N, sizeof(double));
                A->f[k] = (double *)calloc(N, sizeof(double));
                A->v[k] = (double *)calloc(N, sizeof(double));
            }
            A->r[k] = (double *)calloc(N, sizeof(double));
        }
        if (scheme == 2) {
            if (l == 0) {
                A->phik = (double *)phik;
            } else {
                A->phik = (double *)calloc(N, sizeof(double));
                orc_restrict(H.L[l - 1].m, H.L[l - 1].n, H.L[l - 1].phik, A->phik);
            }
        } else {
            A->phik = NULL;
        }
        if (!pin) {
            A->pin = NULL;
        } else if (l == 0) {
            A->pin = (double *)pin;
        } else {
            A->pin = (double *)calloc(N, sizeof(double));
            orc_restrict(H.L[l - 1].m, H.L[l - 1].n, H.L[l - 1].pin, A->pin);
        }
    }
    orc_level *F = &H.L[0];
    orc_residual(scheme, m, n, h, c, alpha, F->phik, phi, mu, ka, S1, S2, S3, F->r[0], F->r[1],
                 F->r[2], F->pin);
    double nr = orc_norm3(m, n, h, F->r[0], F->r[1], F->r[2]);
    history[0] = nr;
    int cyc = 0;
    while (!(nr <= tol) && cyc < max_cycles) {
        if (nlev == 1 && coarse_sweeps > 0) {
            orc_smooth(scheme, newton, coarse_sweeps, m, n, h, c, alpha, F->phik, phi, mu, ka, S1,
                       S2, S3, F->pin);
        } else if (nlev == 1) {
            orc_dense_newton(scheme, m, n, h, c, alpha, F->phik, phi, mu, ka, S1, S2, S3, 50, F->pin);
        } else {
            vcycle(&H, 0);
        }
        ++cyc;
        orc_residual(scheme, m, n, h, c, alpha, F->phik, phi, mu, ka, S1, S2, S3, F->r[0],
                     F->r[1], F->r[2], F->pin);
        nr = orc_norm3(m, n, h, F->r[0], F->r[1], F->r[2]);
        history[cyc] = nr;
        if (!isfinite(nr)) break;
    }
    for (int l = 0; l < nlev; ++l) {
        orc_level *A = &H.L[l];
        for (int k = 0; k < 3; ++k) {
            if (l > 0) { free(A->u[k]); free(A->f[k]); free(A->v[k]); }
            free(A->r[k]);
        }
        if (l > 0 && A->phik) free(A->phik);
        if (l > 0 && A->pin) free(A->pin);
    }
    free(H.L);
    return nr <= tol ? cyc : -(cyc + 1);
}

/* ------------------------------------------------------------------------ */
/* Initial guess completion, psi update, energies.                          */
/* ------------------------------------------------------------------------ */

/* Given phi, set kappa and mu so that N^(3) = S^(3) and N^(2) = S^(2) hold
 * exactly: kappa = S3 + e Lap(phi), then mu = S2 + g(phi) + al phi + Lap(kappa). */
void orc_complete_guess(int scheme, int m, int n, double h, double alpha, const double *phik,
                        const double *phi, double *mu, double *ka, const double *S2,
                        const double *S3, const double *pin) {
    double al = alin(scheme, alpha), e = ecoef(scheme);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            size_t q = IX(i, j, m);
            ka[q] = S3[q] + e * lap_at(phi, i, j, m, n, h);
        }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            size_t q = IX(i, j, m);
            double xk = phik ? phik[q] : 0.0;
            double alq = al + (pin ? pin[q] : 0.0);
            mu[q] = S2[q] + gnl(scheme, phi[q], xk) + alq * phi[q] + lap_at(ka, i, j, m, n, h);
        }
}

/* psi^{k+1} from eq. discrete_1_b (scheme 1) or discrete_2_b (scheme 2). */
void orc_psi_update(int scheme, size_t N, double s, const double *phinew, const double *phik,
                    const double *psik, double *psinew) {
    for (size_t q = 0; q < N; ++q) {
        if (scheme == 1)
            psinew[q] = (phinew[q] - phik[q]) / s;
        else
            psinew[q] = (2.0 / s) * (phinew[q] - phik[q]) - (psik ? psik[q] : 0.0);
    }
}

/* Discrete energy F (eq. discrete_energy_PFC):
 * F = 1/4 ||phi||_4^4 + alpha/2 ||phi||_2^2 - ||grad_h phi||_2^2 + 1/2 ||Lap_h phi||_2^2,
 * with ||f||_p^p = h^2 sum |f|^p and ||grad_h f||_2^2 = sum over east and north
 * cell edges of the squared difference (the h^2 weight and 1/h^2 cancel). */
double orc_energy_F(int m, int n, double h, double eps, const double *phi) {
    double alpha = 1.0 - eps, h2 = h * h;
    double s4 = 0.0, s2 = 0.0, sg = 0.0, sl = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            double x = phi[IX(i, j, m)];
            double dx = phi[IX(wrapx(i + 1, m), j, m)] - x;
            double dy = phi[IX(i, wrapy(j + 1, n), m)] - x;
            double L = lap_at(phi, i, j, m, n, h);
            s4 += x * x * x * x;
            s2 += x * x;
            sg += dx * dx + dy * dy;
            sl += L * L;
        }
    return 0.25 * h2 * s4 + 0.5 * alpha * h2 * s2 - sg + 0.5 * h2 * sl;
}

/* ||grad_h f||_2^2 = sum of squared east and north edge differences. */
double orc_grad_sq(int m, int n, const double *f) {
    double sg = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            double x = f[IX(i, j, m)];
            double dx = f[IX(wrapx(i + 1, m), j, m)] - x;
            double dy = f[IX(i, wrapy(j + 1, n), m)] - x;
            sg += dx * dx + dy * dy;
        }
    return sg;
}

/* Solve -Lap_h w = b - mean(b), mean(w) = 0, by conjugate gradients
 * (the operator is symmetric positive definite on mean-zero functions).
 * Iterates until ||residual||_2 <= rtol * ||b - mean(b)||_2.
 * Returns the iteration count (or -1 if maxit was reached). */
int orc_poisson_cg(int m, int n, double h, const double *b, double *w, double rtol, int maxit) {
    size_t N = (size_t)m * n;
    double *r = (double *)malloc(N * sizeof(double));
    double *pp = (double *)malloc(N * sizeof(double));
    double *Ap = (double *)malloc(N * sizeof(double));
    double mean = 0.0;
    for (size_t q = 0; q < N; ++q) mean += b[q];
    mean /= (double)N;
    double bn = 0.0, rr = 0.0;
    for (size_t q = 0; q < N; ++q) {
        w[q] = 0.0;
        r[q] = b[q] - mean;
        pp[q] = r[q];
        bn += r[q] * r[q];
    }
    rr = bn;
    int it = 0, ret = -1;
    if (bn == 0.0) { ret = 0; goto out; }
    for (it = 1; it <= maxit; ++it) {
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i) Ap[IX(i, j, m)] = -lap_at(pp, i, j, m, n, h);
        double pAp = 0.0;
        for (size_t q = 0; q < N; ++q) pAp += pp[q] * Ap[q];
        double a = rr / pAp;
        double rr2 = 0.0;
        for (size_t q = 0; q < N; ++q) {
            w[q] += a * pp[q];
            r[q] -= a * Ap[q];
            rr2 += r[q] * r[q];
        }
        if (sqrt(rr2) <= rtol * sqrt(bn)) { ret = it; break; }
        double beta = rr2 / rr;
        rr = rr2;
        for (size_t q = 0; q < N; ++q) pp[q] = r[q] + beta * pp[q];
    }
out:
    /* remove any drift of the mean */
    {
        double mw = 0.0;
        for (size_t q = 0; q < N; ++q) mw += w[q];
        mw /= (double)N;
        for (size_t q = 0; q < N; ++q) w[q] -= mw;
    }
    free(r); free(pp); free(Ap);
    return ret;
}

/* ||psi||_{-1}^2 = h^2 (psi, w) with -Lap_h w = psi - mean(psi) (App. A,
 * mean-zero space and "-1" norm).  The mean of psi is projected out first. */
double orc_norm_m1_sq(int m, int n, double h, const double *psi) {
    size_t N = (size_t)m * n;
    double *w = (double *)malloc(N * sizeof(double));
    orc_poisson_cg(m, n, h, psi, w, 1e-14, 100000);
    double mean = 0.0;
    for (size_t q = 0; q < N; ++q) mean += psi[q];
    mean /= (double)N;
    double acc = 0.0;
    for (size_t q = 0; q < N; ++q) acc += (psi[q] - mean) * w[q];
    free(w);
    return h * h * acc;
}

/* Energies after a step (Sec. 3): out[0] = F(phi^{k+1}),
 * out[1] = pseudo energy F + ||psi^{k+1}||_{-1}^2 / (2M),
 * out[2] = modified energy pseudo + 1/2 ||grad_h(phi^{k+1} - phi^k)||^2,
 * out[3] = mass h^2 sum phi^{k+1}. */
void orc_energies(int m, int n, double h, double eps, double M, const double *phinew,
                  const double *phik, const double *psinew, double *out, const double *pin,
                  const double *phihat) {
    size_t N = (size_t)m * n;
    double F = orc_energy_F(m, n, h, eps, phinew);
    if (pin) {
        double sp = 0.0;
        for (size_t q = 0; q < N; ++q) {
            double dp = phinew[q] - phihat[q];
            sp += pin[q] * dp * dp;
        }
        F += h * h * sp;
    }
    double nm1 = orc_norm_m1_sq(m, n, h, psinew);
    double *d = (double *)malloc(N * sizeof(double));
    double mass = 0.0;
    for (size_t q = 0; q < N; ++q) {
        d[q] = phinew[q] - phik[q];
        mass += phinew[q];
    }
    double g = orc_grad_sq(m, n, d);
    free(d);
    out[0] = F;
    out[1] = F + nm1 / (2.0 * M);
    out[2] = out[1] + 0.5 * g;
    out[3] = h * h * mass;
}

/* ------------------------------------------------------------------------ */
/* One whole time step.                                                     */
/* ------------------------------------------------------------------------ */

/* Given phi^k, phi^{k-1} (scheme 2; may equal phi^k) and psi^k, compute
 * phi^{k+1}, mu, kappa, psi^{k+1} and the energies.
 * guess: 0 -> phi^{(0)} = phi^k; 1 -> phi^{(0)} = 2 phi^k - phi^{k-1}.
 * Returns the number of V-cycles, or a negative count if tol was not met. */
int orc_step(const orc_model *p, int newton, int m, int n, const double *phik,
             const double *phikm1, const double *psik, int guess, int nu1, int nu2, int coarsest,
             int coarse_sweeps, double tol, int max_cycles, double *phinew, double *mu, double *ka, double *psinew,
             double *history, double *energies, const double *pin, const double *phihat) {
    size_t N = (size_t)m * n;
    double c, d;
    orc_coefficients(p, &c, &d);
    double alpha = 1.0 - p->eps;
    double *S1 = (double *)malloc(N * sizeof(double));
    double *S2 = (double *)malloc(N * sizeof(double));
    double *S3 = (double *)malloc(N * sizeof(double));
    orc_source(p, m, n, phik, phikm1, psik, S1, S2, S3, pin, phihat);
    for (size_t q = 0; q < N; ++q)
        phinew[q] = (guess == 1) ? 2.0 * phik[q] - phikm1[q] : phik[q];
    const double *pk = p->scheme == 2 ? phik : NULL;
    orc_complete_guess(p->scheme, m, n, p->h, alpha, pk, phinew, mu, ka, S2, S3, pin);
    int cyc = orc_fas_solve(p->scheme, newton, m, n, p->h, c, alpha, pk, phinew, mu, ka, S1, S2,
                            S3, nu1, nu2, coarsest, coarse_sweeps, tol, max_cycles, history, pin);
    orc_psi_update(p->scheme, N, p->s, phinew, phik, psik, psinew);
    if (energies) orc_energies(m, n, p->h, p->eps, p->M, phinew, phik, psinew, energies, pin, phihat);
    free(S1); free(S2); free(S3);
    return cyc;
}

int orc_version(void) { return 1; }

/* Number of OpenMP threads the oracle's parallel loops use. */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the OpenMP loops (the CPU timing of the oracle); no effect on
 * the arithmetic. */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
