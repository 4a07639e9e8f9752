// Three-dimensional form of the step: the schemes of Sec. 3.1 / 3.2 and the
// multigrid of App. B with the seven-point Laplacian (the paper notes that the
// extension to three dimensions is straightforward).  Periodic m x n x l grids
// with power-of-two sides, cell (i, j, k) at (k n + j) m + i, FP64.
//
// Kernels are plain global-memory passes, one thread per cell (or per cell of
// one colour): a red-black half-sweep, the residual with the 2x2x2 restriction
// of u, r and phi^k, the completion of a coarse right-hand side, the trilinear
// prolongation and correction, and the residual norm.  Every pass is bound by
// HBM bandwidth; each launch streams its level once.
#pragma once
#include "kernels.hpp"

namespace mpfc {

struct Grid3 {
    int m, n, l;      // cells along x, y, z (powers of two)
    int lm, ln, ll;   // their log2
};

__device__ __forceinline__ size_t at3(int i, int j, int k, const Grid3& g) {
    return ((((size_t)k << g.ln) + (size_t)j) << g.lm) + (size_t)i;
}

// Sum of the six face neighbours (periodic wrap-around).
__device__ __forceinline__ double nsum6(const double* __restrict__ f, int i, int j, int k,
                                        const Grid3& g) {
    const int ip = (i + 1) & (g.m - 1), im = (i - 1) & (g.m - 1);
    const int jp = (j + 1) & (g.n - 1), jm = (j - 1) & (g.n - 1);
    const int kp = (k + 1) & (g.l - 1), km = (k - 1) & (g.l - 1);
    return ((f[at3(ip, j, k, g)] + f[at3(im, j, k, g)]) + (f[at3(i, jp, k, g)] + f[at3(i, jm, k, g)])) +
           (f[at3(i, j, kp, g)] + f[at3(i, j, km, g)]);
}

// MPFC system N(u) = f in three dimensions (App. B.1 / B.2 with the seven-point
// Laplacian): the same algebra as in two dimensions with the centre weight 6.
template <int SCHEME, bool NEWTON>
struct MpfcOp3 {
    static constexpr int NF = 3;
    static constexpr bool XK = SCHEME == 2;
    LevelOp<double> op;
    __device__ __forceinline__ void apply(const double* u, const double* ns, double xk,
                                          double* N) const {
        const double lphi = (ns[0] - 6.0 * u[0]) * op.ih2;
        const double lmu = (ns[1] - 6.0 * u[1]) * op.ih2;
        const double lka = (ns[2] - 6.0 * u[2]) * op.ih2;
        N[0] = u[0] - op.c * lmu;
        N[1] = u[1] - nl_value<double, SCHEME, false>(u[0], 0.0, xk) - op.al * u[0] - lka;
        N[2] = u[2] - op.e * lphi;
    }
    // J_loc delta = f - N(u), J_loc = [[1, a, 0], [-d, 1, b], [ec, 0, 1]] with
    // a = 6c/h^2, b = 6/h^2, ec = 6e/h^2, d = al + g'(phi) (Newton) or Picard's.
    __device__ __forceinline__ void relax(double* u, const double* ns, const double* f,
                                          double xk) const {
        double N[3];
        apply(u, ns, xk, N);
        const double r1 = f[0] - N[0], r2 = f[1] - N[1], r3 = f[2] - N[2];
        const double d = op.al + nl_lin<double, SCHEME, NEWTON>(u[0], xk);
        const double a = 6.0 * op.c * op.ih2, b = 6.0 * op.ih2, ec = 6.0 * op.e * op.ih2;
        const double det = 1.0 + a * d + a * b * ec;
        const double dm = (r2 + (d + b * ec) * r1 - b * r3) / det;
        const double dx = r1 - a * dm;
        const double dk = r3 - ec * dx;
        u[0] += dx;
        u[1] += dm;
        u[2] += dk;
    }
};

// Poisson problem -Lap_h w = b of the -1 norm, same interface.
struct PoissonOp3 {
    static constexpr int NF = 1;
    static constexpr bool XK = false;
    double ih2, h2;
    __device__ __forceinline__ void apply(const double* u, const double* ns, double,
                                          double* N) const {
        N[0] = (6.0 * u[0] - ns[0]) * ih2;
    }
    __device__ __forceinline__ void relax(double* u, const double* ns, const double* f,
                                          double) const {
        u[0] = (h2 * f[0] + ns[0]) / 6.0;
    }
};

// Fields of one level.
struct L3 {
    double* u[3];
    const double* f[3];
    const double* xk;   // phi^k on this level (scheme 2)
};

// One half-sweep: every cell of colour `colour` ((i + j + k) even = 0, red).
// Cells of one colour only read the other colour, so the update is in place.
template <class Op>
__global__ void __launch_bounds__(256) k3_relax(Op op, Grid3 g, L3 A, int colour,
                                                const CycleState* st) {
    if (stopped(st)) return;
    const size_t half = ((size_t)g.m * g.n * g.l) >> 1;
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= half) return;
    const int ii = (int)(t & (size_t)((g.m >> 1) - 1));
    const size_t r = t >> (g.lm - 1);
    const int j = (int)(r & (size_t)(g.n - 1)), k = (int)(r >> g.ln);
    const int i = 2 * ii + ((j + k + colour) & 1);
    const size_t q = at3(i, j, k, g);
    constexpr int NF = Op::NF;
    double u[NF], ns[NF], fv[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        u[f] = A.u[f][q];
        ns[f] = nsum6(A.u[f], i, j, k, g);
        fv[f] = A.f[f][q];
    }
    op.relax(u, ns, fv, Op::XK ? A.xk[q] : 0.0);
#pragma unroll
    for (int f = 0; f < NF; ++f) A.u[f][q] = u[f];
}

// Residual r = f - N(u) at the eight fine cells of each coarse cell and the
// 2x2x2 averages of u (into uH and vH), r (rH) and, if xkH is set, phi^k.
// One thread per coarse cell; g is the fine grid.
template <class Op>
__global__ void __launch_bounds__(256) k3_restrict(Op op, Grid3 g, L3 A, L3 H, double* vH0,
                                                   double* vH1, double* vH2, double* rH0,
                                                   double* rH1, double* rH2, double* xkH,
                                                   const CycleState* st) {
    if (stopped(st)) return;
    const Grid3 c{g.m >> 1, g.n >> 1, g.l >> 1, g.lm - 1, g.ln - 1, g.ll - 1};
    const size_t Q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (Q >= (size_t)c.m * c.n * c.l) return;
    const int I = (int)(Q & (size_t)(c.m - 1));
    const int J = (int)((Q >> c.lm) & (size_t)(c.n - 1));
    const int K = (int)(Q >> (c.lm + c.ln));
    constexpr int NF = Op::NF;
    double su[NF], sr[NF], sxk = 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f) { su[f] = 0.0; sr[f] = 0.0; }
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
        const int i = 2 * I + (cc & 1), j = 2 * J + ((cc >> 1) & 1), k = 2 * K + (cc >> 2);
        const size_t q = at3(i, j, k, g);
        double u[NF], ns[NF], N[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            u[f] = A.u[f][q];
            ns[f] = nsum6(A.u[f], i, j, k, g);
        }
        const double xk = Op::XK ? A.xk[q] : 0.0;
        op.apply(u, ns, xk, N);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            su[f] += u[f];
            sr[f] += A.f[f][q] - N[f];
        }
        sxk += xk;
    }
    double* vH[3] = {vH0, vH1, vH2};
    double* rH[3] = {rH0, rH1, rH2};
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        H.u[f][Q] = 0.125 * su[f];
        vH[f][Q] = 0.125 * su[f];
        rH[f][Q] = 0.125 * sr[f];
    }
    if (Op::XK && xkH) xkH[Q] = 0.125 * sxk;
}

// Coarse right-hand side of the FAS: fout = R r + N(u) with u the restricted
// iterate (A.f holds R r).
template <class Op>
__global__ void __launch_bounds__(256) k3_complete(Op op, Grid3 g, L3 A, double* f0, double* f1,
                                                   double* f2, const CycleState* st) {
    if (stopped(st)) return;
    const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= (size_t)g.m * g.n * g.l) return;
    const int i = (int)(q & (size_t)(g.m - 1));
    const int j = (int)((q >> g.lm) & (size_t)(g.n - 1));
    const int k = (int)(q >> (g.lm + g.ln));
    constexpr int NF = Op::NF;
    double u[NF], ns[NF], N[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        u[f] = A.u[f][q];
        ns[f] = nsum6(A.u[f], i, j, k, g);
    }
    op.apply(u, ns, Op::XK ? A.xk[q] : 0.0, N);
    double* fo[3] = {f0, f1, f2};
#pragma unroll
    for (int f = 0; f < NF; ++f) fo[f][q] = A.f[f][q] + N[f];
}

// u += trilinear interpolation of (uH - vH): per axis 3/4 of the parent's
// coarse index and 1/4 of the coarse neighbour on the fine cell's side.  One
// thread per fine cell; g is the fine grid.
template <int NF>
__global__ void __launch_bounds__(256) k3_prolong(Grid3 g, L3 A, L3 H, const double* vH0,
                                                  const double* vH1, const double* vH2,
                                                  const CycleState* st) {
    if (stopped(st)) return;
    const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= (size_t)g.m * g.n * g.l) return;
    const int i = (int)(q & (size_t)(g.m - 1));
    const int j = (int)((q >> g.lm) & (size_t)(g.n - 1));
    const int k = (int)(q >> (g.lm + g.ln));
    const Grid3 c{g.m >> 1, g.n >> 1, g.l >> 1, g.lm - 1, g.ln - 1, g.ll - 1};
    const int I[2] = {i >> 1, ((i >> 1) + ((i & 1) ? 1 : -1)) & (c.m - 1)};
    const int J[2] = {j >> 1, ((j >> 1) + ((j & 1) ? 1 : -1)) & (c.n - 1)};
    const int K[2] = {k >> 1, ((k >> 1) + ((k & 1) ? 1 : -1)) & (c.l - 1)};
    const double w[2] = {0.75, 0.25};
    const double* vH[3] = {vH0, vH1, vH2};
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        double v = 0.0;
#pragma unroll
        for (int z = 0; z < 2; ++z)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int x = 0; x < 2; ++x) {
                    const size_t Q = at3(I[x], J[y], K[z], c);
                    v += w[x] * w[y] * w[z] * (H.u[f][Q] - vH[f][Q]);
                }
        A.u[f][q] += v;
    }
}

// Per-block sums of r^2 = (f - N(u))^2 over all fields (the stopping test;
// k_norm_finalize / k_p_finalize turn them into the norm).
template <class Op, int NT>
__global__ void __launch_bounds__(NT) k3_resnorm(Op op, Grid3 g, L3 A, double* part,
                                                 const CycleState* st) {
    if (stopped(st)) return;
    __shared__ double red[NT / 64];
    double acc = 0.0;
    const size_t total = (size_t)g.m * g.n * g.l;
    constexpr int NF = Op::NF;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        const int i = (int)(q & (size_t)(g.m - 1));
        const int j = (int)((q >> g.lm) & (size_t)(g.n - 1));
        const int k = (int)(q >> (g.lm + g.ln));
        double u[NF], ns[NF], N[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            u[f] = A.u[f][q];
            ns[f] = nsum6(A.u[f], i, j, k, g);
        }
        op.apply(u, ns, Op::XK ? A.xk[q] : 0.0, N);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const double r = A.f[f][q] - N[f];
            acc += r * r;
        }
    }
    const double bs = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

// ---- per-step passes ----------------------------------------------------------
// Source S (App. B.1 / B.2) with the seven-point Laplacian.
template <int SCHEME>
__global__ void __launch_bounds__(256) k3_source(Grid3 g, double ih2, double d, double alpha,
                                                 const double* __restrict__ phik,
                                                 const double* __restrict__ phikm1,
                                                 const double* __restrict__ psik, double* S1,
                                                 double* S2, double* S3) {
    const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= (size_t)g.m * g.n * g.l) return;
    const int i = (int)(q & (size_t)(g.m - 1));
    const int j = (int)((q >> g.lm) & (size_t)(g.n - 1));
    const int k = (int)(q >> (g.lm + g.ln));
    const double x = phik[q];
    const double lk = (nsum6(phik, i, j, k, g) - 6.0 * x) * ih2;
    S1[q] = x + d * psik[q];
    if constexpr (SCHEME == 1) {
        S2[q] = 2.0 * lk;
        S3[q] = 0.0;
    } else {
        // Lap of phi~ = (3 phi^k - phi^{k-1})/2 from the two Laplacians
        const double lm1 = (nsum6(phikm1, i, j, k, g) - 6.0 * phikm1[q]) * ih2;
        S2[q] = 0.5 * alpha * x + 2.0 * (0.5 * (3.0 * lk - lm1));
        S3[q] = 0.5 * lk;
    }
}

// kappa = S3 + e Lap phi (completion of the guess, first half).
__global__ void __launch_bounds__(256) k3_complete_kappa(Grid3 g, double ih2, double e,
                                                         const double* __restrict__ phi,
                                                         const double* __restrict__ S3,
                                                         double* ka) {
    const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= (size_t)g.m * g.n * g.l) return;
    const int i = (int)(q & (size_t)(g.m - 1));
    const int j = (int)((q >> g.lm) & (size_t)(g.n - 1));
    const int k = (int)(q >> (g.lm + g.ln));
    ka[q] = S3[q] + e * ((nsum6(phi, i, j, k, g) - 6.0 * phi[q]) * ih2);
}

// mu = S2 + g(phi) + al phi + Lap kappa (second half).
template <int SCHEME>
__global__ void __launch_bounds__(256) k3_complete_mu(Grid3 g, double ih2, double al,
                                                      const double* __restrict__ phi,
                                                      const double* __restrict__ phik,
                                                      const double* __restrict__ S2,
                                                      const double* __restrict__ ka, double* mu) {
    const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= (size_t)g.m * g.n * g.l) return;
    const int i = (int)(q & (size_t)(g.m - 1));
    const int j = (int)((q >> g.lm) & (size_t)(g.n - 1));
    const int k = (int)(q >> (g.lm + g.ln));
    const double x = phi[q];
    mu[q] = S2[q] + nl_value<double, SCHEME, false>(x, 0.0, SCHEME == 2 ? phik[q] : 0.0) +
            al * x + (nsum6(ka, i, j, k, g) - 6.0 * ka[q]) * ih2;
}

// phi^(0) = phi^k (mode 0) or 2 phi^k - phi^{k-1} (mode 1).
__global__ void __launch_bounds__(256) k3_guess(size_t total, int mode,
                                                const double* __restrict__ phik,
                                                const double* __restrict__ phikm1, double* phi) {
    const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= total) return;
    phi[q] = mode == 1 ? 2.0 * phik[q] - phikm1[q] : phik[q];
}

// b = psi - mean(psi) (mean from psisum[0]); per-block sums of b^2 and, with a
// warm start w, of (b + Lap_h w)^2 into part[2 blk], part[2 blk + 1].
template <int NT>
__global__ void __launch_bounds__(NT) k3_p_rhs(Grid3 g, double ih2, const double* __restrict__ psi,
                                               const double* __restrict__ psisum, double* b,
                                               const double* __restrict__ w, double* part) {
    __shared__ double red[NT / 64];
    const size_t total = (size_t)g.m * g.n * g.l;
    const double mean = psisum[0] / (double)total;
    double sb = 0.0, sr = 0.0;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        const double v = psi[q] - mean;
        b[q] = v;
        sb += v * v;
        if (w) {
            const int i = (int)(q & (size_t)(g.m - 1));
            const int j = (int)((q >> g.lm) & (size_t)(g.n - 1));
            const int k = (int)(q >> (g.lm + g.ln));
            const double r = v - (6.0 * w[q] - nsum6(w, i, j, k, g)) * ih2;
            sr += r * r;
        }
    }
    const double tb = block_sum<NT>(sb, red);
    __syncthreads();
    const double tr = block_sum<NT>(sr, red);
    if (threadIdx.x == 0) {
        part[(size_t)blockIdx.x * 2] = tb;
        part[(size_t)blockIdx.x * 2 + 1] = tr;
    }
}

// Energy sums, per block into part[blk * 8 + k]: 0: sum phi^4, 1: sum phi^2,
// 2: sum over east/north/top faces of (phi difference)^2, 3: sum (Lap_h phi)^2,
// 4: sum phi, 5: face sum of (difference of phi - phi_prev)^2, 6: sum b w, 7: 0.
template <int NT>
__global__ void __launch_bounds__(NT) k3_energy_terms(Grid3 g, double ih2,
                                                      const double* __restrict__ phi,
                                                      const double* __restrict__ phiprev,
                                                      const double* __restrict__ b,
                                                      const double* __restrict__ w, double* part) {
    __shared__ double red[NT / 64];
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const size_t total = (size_t)g.m * g.n * g.l;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        const int i = (int)(q & (size_t)(g.m - 1));
        const int j = (int)((q >> g.lm) & (size_t)(g.n - 1));
        const int k = (int)(q >> (g.lm + g.ln));
        const size_t qe = at3((i + 1) & (g.m - 1), j, k, g);
        const size_t qn = at3(i, (j + 1) & (g.n - 1), k, g);
        const size_t qt = at3(i, j, (k + 1) & (g.l - 1), g);
        const double x = phi[q];
        const double L = (nsum6(phi, i, j, k, g) - 6.0 * x) * ih2;
        a[0] += (x * x) * (x * x);
        a[1] += x * x;
        a[2] += (phi[qe] - x) * (phi[qe] - x) + (phi[qn] - x) * (phi[qn] - x) +
                (phi[qt] - x) * (phi[qt] - x);
        a[3] += L * L;
        a[4] += x;
        if (phiprev) {
            const double d = x - phiprev[q];
            const double de = phi[qe] - phiprev[qe] - d;
            const double dn = phi[qn] - phiprev[qn] - d;
            const double dt = phi[qt] - phiprev[qt] - d;
            a[5] += de * de + dn * dn + dt * dt;
        }
        a[6] += b[q] * w[q];
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const double t = block_sum<NT>(a[s], red);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * 8 + s] = t;
        __syncthreads();
    }
}

}  // namespace mpfc
