// Per-step kernels of the MPFC time step on gfx950 (one thread per cell, or
// grid-stride reductions): the finest-grid residual norm, the FP64 defect of
// mixed precision, the source S, the initial guess and its completion, the
// 2x2 average and the psi update.  The cell operators and types they use are
// in kernels.hpp.
#pragma once
#include "kernels.hpp"

namespace mpfc {

// Finest-grid residual sum of squares sum_c sum_ij r_c^2 (FP64, the stopping
// test; k_norm_finalize turns the per-block sums into the norm).  With r0
// non-null the residual is also stored.
template <int SCHEME, int NT>
__global__ void __launch_bounds__(NT) k_resnorm(Fields<double> F, LevelOp<double> op, Grid g,
                                                const CycleState* st, double* part, double* r0,
                                                double* r1o, double* r2o) {
    if (stopped(st)) return;
    __shared__ double red[NT / 64];
    double acc = 0.0;
    const size_t total = (size_t)g.m * g.n;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        int i, j;
        cell_of(q, g, i, j);
        double a, b, c;
        residual_at<double, SCHEME, false>(F, op, g, i, j, a, b, c);
        acc += a * a + b * b + c * c;
        if (r0) { r0[q] = a; r1o[q] = b; r2o[q] = c; }
    }
    const double bs = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;  // summed by k_norm_finalize
}

// Mixed precision, outer FP64 defect-correction step on the finest grid, one
// cell: u_new = u + e (the FP32 correction; `add` = 0 keeps u, for the first
// residual of a step), r = S - N(u_new) in FP64, and the inputs of the next
// FP32 correction solve: r rounded to FP32 and the base phi rounded to FP32.
// The neighbours' u + e are recomputed here, so no other thread's write is
// read.  Returns the cell's sum of squared residuals (the stopping test).
template <int SCHEME>
__device__ __forceinline__ double defect_cell(const Fields<double>& F, const LevelOp<double>& op,
                                              const Grid& g, const float* __restrict__ e0,
                                              const float* __restrict__ e1,
                                              const float* __restrict__ e2, int add, double* un0,
                                              double* un1, double* un2, float* r0, float* r1,
                                              float* r2, float* pbase, int i, int j) {
    const size_t q = at(i, j, g);
    const size_t nb[4] = {at(wrapx(i + 1, g), j, g), at(wrapx(i - 1, g), j, g),
                          at(i, wrapy(j + 1, g), g), at(i, wrapy(j - 1, g), g)};
    auto val = [&](const double* u, const float* e, size_t k) {
        return add ? u[k] + (double)e[k] : u[k];
    };
    const double x = val(F.phi, e0, q), y = val(F.mu, e1, q), z = val(F.ka, e2, q);
    double sx = 0, sy = 0, sz = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        sx += val(F.phi, e0, nb[k]);
        sy += val(F.mu, e1, nb[k]);
        sz += val(F.ka, e2, nb[k]);
    }
    const double xk = SCHEME == 2 ? F.phik[q] : 0.0;
    const double lphi = (sx - 4.0 * x) * op.ih2;
    const double lmu = (sy - 4.0 * y) * op.ih2;
    const double lka = (sz - 4.0 * z) * op.ih2;
    const double a = F.f1[q] - (x - op.c * lmu);
    const double b = F.f2[q] - (y - nl_value<double, SCHEME, false>(x, 0.0, xk) - op.al * x - lka);
    const double c = F.f3[q] - (z - op.e * lphi);
    un0[q] = x; un1[q] = y; un2[q] = z;
    r0[q] = (float)a; r1[q] = (float)b; r2[q] = (float)c;
    pbase[q] = (float)x;
    return a * a + b * b + c * c;
}

// The same on a 32 x 8 tile per workgroup (one cell per thread): u + e of the
// tile and a ring of one cell (the neighbour rule of wrapx / wrapy) is formed
// once into LDS, so each cell's value is loaded from memory once instead of
// by its five stencils.  Same arithmetic and order per cell as defect_cell;
// per-block sums of r^2 into part[] (blockIdx.y * gridDim.x + blockIdx.x),
// summed by k_norm_finalize.  The correction e is cleared by the next outer
// iteration, not here (other workgroups still read it for their ring).
constexpr int DT_X = 32, DT_Y = 8;
template <int SCHEME>
__global__ void __launch_bounds__(DT_X * DT_Y) k_defect_tile(Fields<double> F, LevelOp<double> op,
                                                            Grid g, const CycleState* st,
                                                            double* part,
                                                            const float* __restrict__ e0,
                                                            const float* __restrict__ e1,
                                                            const float* __restrict__ e2, int add,
                                                            double* un0, double* un1, double* un2,
                                                            float* r0, float* r1, float* r2,
                                                            float* pbase) {
    constexpr int NT = DT_X * DT_Y, LX = DT_X + 2, LY = DT_Y + 2, NL = LX * LY;
    if (stopped(st)) return;
    __shared__ double U[3][LY][LX];
    __shared__ double red[NT / 64];
    const int t = threadIdx.x;
    const int x0 = blockIdx.x * DT_X, y0 = blockIdx.y * DT_Y;
    // tile + ring: every load issued before the LDS stores (indices clamped)
    constexpr int NR = (NL + NT - 1) / NT;
    double v[NR][3];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int c = min(t + k * NT, NL - 1);
        const int ly = c / LX, lx = c - ly * LX;
        const int gi = wrapx(min(max(x0 + lx - 1, -1), g.m), g);
        const int gj = wrapy(min(max(y0 + ly - 1, -1), g.n), g);
        const size_t q = at(gi, gj, g);
        v[k][0] = add ? F.phi[q] + (double)e0[q] : F.phi[q];
        v[k][1] = add ? F.mu[q] + (double)e1[q] : F.mu[q];
        v[k][2] = add ? F.ka[q] + (double)e2[q] : F.ka[q];
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int c = t + k * NT;
        if (c < NL) {
            const int ly = c / LX, lx = c - ly * LX;
            U[0][ly][lx] = v[k][0];
            U[1][ly][lx] = v[k][1];
            U[2][ly][lx] = v[k][2];
        }
    }
    __syncthreads();
    const int tx = t % DT_X, ty = t / DT_X;
    const int i = x0 + tx, j = y0 + ty;
    double acc = 0.0;
    if (i < g.m && j < g.n) {
        const size_t q = at(i, j, g);
        const int lx = tx + 1, ly = ty + 1;
        const double x = U[0][ly][lx], y = U[1][ly][lx], z = U[2][ly][lx];
        // neighbours in defect_cell's order: east, west, north, south
        const double sx = ((U[0][ly][lx + 1] + U[0][ly][lx - 1]) + U[0][ly + 1][lx]) + U[0][ly - 1][lx];
        const double sy = ((U[1][ly][lx + 1] + U[1][ly][lx - 1]) + U[1][ly + 1][lx]) + U[1][ly - 1][lx];
        const double sz = ((U[2][ly][lx + 1] + U[2][ly][lx - 1]) + U[2][ly + 1][lx]) + U[2][ly - 1][lx];
        const double xk = SCHEME == 2 ? F.phik[q] : 0.0;
        const double lphi = (sx - 4.0 * x) * op.ih2;
        const double lmu = (sy - 4.0 * y) * op.ih2;
        const double lka = (sz - 4.0 * z) * op.ih2;
        const double a = F.f1[q] - (x - op.c * lmu);
        const double b = F.f2[q] - (y - nl_value<double, SCHEME, false>(x, 0.0, xk) - op.al * x - lka);
        const double c = F.f3[q] - (z - op.e * lphi);
        un0[q] = x; un1[q] = y; un2[q] = z;
        r0[q] = (float)a; r1[q] = (float)b; r2[q] = (float)c;
        pbase[q] = (float)x;
        acc = a * a + b * b + c * c;
    }
    const double bs = block_sum<NT>(acc, red);
    if (t == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = bs;
}


template <typename TI, typename TO>
__global__ void __launch_bounds__(256) k_convert(const TI* __restrict__ a, TO* b, size_t n) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) b[q] = (TO)a[q];
}

__global__ void k_state_reset(CycleState* st) {
    if (threadIdx.x == 0) {
        st->acc = 0.0; st->blocks = 0u; st->count = 0;
        st->status = ST_RUNNING; st->done = 0; st->pad0 = st->pad1 = 0;
    }
}

// ---------------------------------------------------------------------------
// Step set-up and wrap-up kernels (one thread per cell).

// Source S (App. B.1 / B.2) at cell (i, j).  d = weight of psi^k.  With the
// pinning of Sec. 4.6 (scheme 2; pin != null) S^(2) gains W (phi^k - 2 phi_hat):
// the unknown mu is then mu~ = mu + 2 ((phi^{k+1} + phi^k)/2 - phi_hat) W.
template <int SCHEME>
__device__ __forceinline__ void source_cell(const Grid& g, double ih2, double d, double alpha,
                                            const double* __restrict__ phik,
                                            const double* __restrict__ phikm1,
                                            const double* __restrict__ psik, double* S1,
                                            double* S2, double* S3, double* phik_copy, int i,
                                            int j, const double* __restrict__ pin = nullptr,
                                            const double* __restrict__ phihat = nullptr) {
    const size_t q = at(i, j, g);
    const double pk = phik[q];
    if (phik_copy) phik_copy[q] = pk;
    const double lk = (nsum(phik, i, j, g) - 4.0 * pk) * ih2;
    S1[q] = pk + d * psik[q];
    if constexpr (SCHEME == 1) {
        S2[q] = 2.0 * lk;
        S3[q] = 0.0;
    } else {
        // 2 Lap((3 phi^k - phi^{k-1})/2) = 3 Lap phi^k - Lap phi^{k-1}
        const double lkm1 = (nsum(phikm1, i, j, g) - 4.0 * phikm1[q]) * ih2;
        S2[q] = 0.5 * alpha * pk + (3.0 * lk - lkm1);
        if (pin) S2[q] += pin[q] * (pk - 2.0 * phihat[q]);
        S3[q] = 0.5 * lk;
    }
}

// Caller arrays of one step.  The step's set-up and wrap-up run as captured
// graphs, so these pointers, which change from step to step, are read from a
// small device table that k_set_io fills before each step.
struct StepIO {
    const double* phi_n;    // phi^k
    const double* phi_nm1;  // phi^{k-1}
    double* psi;            // psi^k on entry, psi^{k+1} after the wrap-up
    double* phi_np1;        // phi^{k+1}
    double* mu;             // optional mu^{k+1} output (null: not asked for)
    double* kappa;          // optional kappa^{k+1} output (null: not asked for)
};

template <int SCHEME>
__global__ void __launch_bounds__(256) k_source(Grid g, double ih2, double d, double alpha,
                                                const double* __restrict__ phik,
                                                const double* __restrict__ phikm1,
                                                const double* __restrict__ psik, double* S1,
                                                double* S2, double* S3, double* phik_copy,
                                                const double* __restrict__ pin,
                                                const double* __restrict__ phihat) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.m || j >= g.n) return;
    source_cell<SCHEME>(g, ih2, d, alpha, phik, phikm1, psik, S1, S2, S3, phik_copy, i, j, pin,
                        phihat);
}

// The same, for a step whose phi^k, phi^{k-1}, psi^k are the caller's arrays
// in `io`.
template <int SCHEME>
__global__ void __launch_bounds__(256) k_source_io(Grid g, double ih2, double d, double alpha,
                                                   const StepIO* __restrict__ io, double* S1,
                                                   double* S2, double* S3, double* phik_copy,
                                                   const double* __restrict__ pin,
                                                   const double* __restrict__ phihat) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.m || j >= g.n) return;
    source_cell<SCHEME>(g, ih2, d, alpha, io->phi_n, io->phi_nm1, io->psi, S1, S2, S3, phik_copy,
                        i, j, pin, phihat);
}

// Initial guess phi^(0): phi^k (mode 0) or 2 phi^k - phi^{k-1} (mode 1).
__device__ __forceinline__ double guess_value(int mode, double pk, double pkm1) {
    return mode == 1 ? 2.0 * pk - pkm1 : pk;
}

// The guess from the caller's arrays in `io`.
__global__ void __launch_bounds__(256) k_guess(Grid g, int mode, const StepIO* __restrict__ io,
                                               double* phi) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (size_t)g.m * g.n) return;
    phi[q] = guess_value(mode, io->phi_n[q], io->phi_nm1[q]);
}

// Consistent completion of the guess: kappa = S3 + e Lap phi (so N^(3) = S^(3)).
__device__ __forceinline__ void complete_kappa_cell(const Grid& g, double ih2, double e,
                                                    const double* __restrict__ phi,
                                                    const double* __restrict__ S3, double* ka,
                                                    int i, int j) {
    const size_t q = at(i, j, g);
    ka[q] = S3[q] + e * (nsum(phi, i, j, g) - 4.0 * phi[q]) * ih2;
}

__global__ void k_set_io(StepIO* io, const double* phi_n, const double* phi_nm1, double* psi,
                         double* phi_np1, double* mu, double* kappa) {
    if (threadIdx.x == 0) {
        io->phi_n = phi_n;
        io->phi_nm1 = phi_nm1;
        io->psi = psi;
        io->phi_np1 = phi_np1;
        io->mu = mu;
        io->kappa = kappa;
    }
}

// Step set-up in one pass (extrapolated or previous-step guess; the caller's
// phi^k, phi^{k-1} and psi^k from `io`): the source S (source_cell), the guess phi0 = guess_value(mode, phi^k, phi^{k-1}) and
// kappa = S3 + e Lap phi0, the first half of the guess's completion.  Each
// thread forms the guess at its four neighbours itself, so no other thread's
// output is read; the arithmetic is that of k_guess and complete_kappa_cell.
// Workgroup (0, 0) also resets the cycle state.
template <int SCHEME>
__global__ void __launch_bounds__(256) k_setup(Grid g, double ih2, double d, double alpha,
                                               double e, int mode,
                                               const StepIO* __restrict__ io, double* S1,
                                               double* S2, double* S3, double* phik_copy,
                                               const double* __restrict__ pin,
                                               const double* __restrict__ phihat, double* phi0,
                                               double* ka, CycleState* st) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && threadIdx.y == 0) {
        st->acc = 0.0; st->blocks = 0u; st->count = 0;
        st->status = ST_RUNNING; st->done = 0; st->pad0 = st->pad1 = 0;
    }
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.m || j >= g.n) return;
    const double* phik = io->phi_n;
    const double* phikm1 = io->phi_nm1;
    source_cell<SCHEME>(g, ih2, d, alpha, phik, phikm1, io->psi, S1, S2, S3, phik_copy, i, j, pin,
                        phihat);
    const size_t q = at(i, j, g);
    auto gv = [&](size_t k) { return guess_value(mode, phik[k], phikm1[k]); };
    const double x = gv(q);
    phi0[q] = x;
    const int ip = wrapx(i + 1, g), im = wrapx(i - 1, g);
    const int jp = wrapy(j + 1, g), jm = wrapy(j - 1, g);
    const double ns = (gv(at(ip, j, g)) + gv(at(im, j, g))) + (gv(at(i, jp, g)) + gv(at(i, jm, g)));
    ka[q] = S3[q] + e * (ns - 4.0 * x) * ih2;
}

// The step's whole set-up on a 32 x 8 tile per workgroup: the source S, the
// guess, kappa and mu (k_setup, then k_complete_mu) and, with NORM, the
// per-block sums of r1^2 of the completed guess (k_resnorm_guess).  phi^k and
// phi^{k-1} of the tile and a ring of three cells (the neighbour rule of
// wrapx / wrapy; reflected rings of a Neumann axis give the mirrored cells'
// values, so kappa and mu there are the mirrored cells' too) are staged in
// LDS; the guess is formed on all of it, kappa on the tile and two rings, mu
// on the tile and one ring.  Same arithmetic and order per cell as those
// kernels.  Sides must be multiples of 32 (x) and 8 (y), at least 32 x 8.
// Workgroup (0, 0) also resets the cycle state.
constexpr int SU_X = 32, SU_Y = 8, SU_H = 3;
template <int SCHEME, bool NORM>
__global__ void __launch_bounds__(SU_X * SU_Y) k_setup_tile(
    Grid g, LevelOp<double> op, double d, double alpha, int mode, const StepIO* __restrict__ io,
    double* S1, double* S2, double* S3, double* phik_copy, const double* __restrict__ pin,
    const double* __restrict__ phihat, double* phi0, double* ka, double* mu, CycleState* st,
    double* part) {
    constexpr int NT = SU_X * SU_Y, LX = SU_X + 2 * SU_H, LY = SU_Y + 2 * SU_H;
    __shared__ double PK[LY][LX], PM[LY][LX], G0[LY][LX], K[LY][LX], MU[LY][LX];
    __shared__ double red[NT / 64];
    const int t = threadIdx.x;
    if (blockIdx.x == 0 && blockIdx.y == 0 && t == 0) {
        st->acc = 0.0; st->blocks = 0u; st->count = 0;
        st->status = ST_RUNNING; st->done = 0; st->pad0 = st->pad1 = 0;
    }
    const int xb = blockIdx.x * SU_X - SU_H, yb = blockIdx.y * SU_Y - SU_H;
    const double* __restrict__ phik = io->phi_n;
    const double* __restrict__ phikm1 = io->phi_nm1;
    const double ih2 = op.ih2;
    // phi^k, phi^{k-1} and the guess on the tile and three rings
    {
        constexpr int NL = LX * LY, NR = (NL + NT - 1) / NT;
        double vk[NR], vm[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int c = min(t + r * NT, NL - 1);
            const int ly = c / LX, lx = c - ly * LX;
            const size_t q = at(wrapx(xb + lx, g), wrapy(yb + ly, g), g);
            vk[r] = phik[q];
            vm[r] = phikm1[q];
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int c = t + r * NT;
            if (c < NL) {
                const int ly = c / LX, lx = c - ly * LX;
                PK[ly][lx] = vk[r];
                PM[ly][lx] = vm[r];
                G0[ly][lx] = guess_value(mode, vk[r], vm[r]);
            }
        }
    }
    __syncthreads();
    auto ns = [&](const double (&A)[LY][LX], int lx, int ly) {
        return (A[ly][lx + 1] + A[ly][lx - 1]) + (A[ly + 1][lx] + A[ly - 1][lx]);
    };
    // kappa = S3 + e Lap phi0 on the tile and two rings
    for (int c = t; c < (LX - 2) * (LY - 2); c += NT) {
        const int ly = 1 + c / (LX - 2), lx = 1 + c % (LX - 2);
        const double lk = (ns(PK, lx, ly) - 4.0 * PK[ly][lx]) * ih2;
        const double s3 = SCHEME == 1 ? 0.0 : 0.5 * lk;
        K[ly][lx] = s3 + op.e * (ns(G0, lx, ly) - 4.0 * G0[ly][lx]) * ih2;
    }
    __syncthreads();
    // S2 of a cell (source_cell's arithmetic)
    auto s2_at = [&](int lx, int ly, size_t q) {
        const double pk = PK[ly][lx];
        const double lk = (ns(PK, lx, ly) - 4.0 * pk) * ih2;
        if constexpr (SCHEME == 1) {
            return 2.0 * lk;
        } else {
            const double lkm1 = (ns(PM, lx, ly) - 4.0 * PM[ly][lx]) * ih2;
            double v = 0.5 * alpha * pk + (3.0 * lk - lkm1);
            if (pin) v += pin[q] * (pk - 2.0 * phihat[q]);
            return v;
        }
    };
    // mu = S2 + g(phi0) + al phi0 + Lap kappa on the tile and one ring
    for (int c = t; c < (LX - 4) * (LY - 4); c += NT) {
        const int ly = 2 + c / (LX - 4), lx = 2 + c % (LX - 4);
        const size_t q = at(wrapx(xb + lx, g), wrapy(yb + ly, g), g);
        const double x = G0[ly][lx];
        const double xk = SCHEME == 2 ? PK[ly][lx] : 0.0;
        const double alq = op.al + (pin ? pin[q] : 0.0);
        MU[ly][lx] = s2_at(lx, ly, q) + nl_value<double, SCHEME, false>(x, 0.0, xk) + alq * x +
                     (ns(K, lx, ly) - 4.0 * K[ly][lx]) * ih2;
    }
    __syncthreads();
    // the tile: S, phi^k copy, guess, kappa, mu and the first residual component
    const int tx = t % SU_X, ty = t / SU_X, lx = tx + SU_H, ly = ty + SU_H;
    const size_t q = at(blockIdx.x * SU_X + tx, blockIdx.y * SU_Y + ty, g);
    const double pk = PK[ly][lx];
    const double s1 = pk + d * io->psi[q];
    S1[q] = s1;
    S2[q] = s2_at(lx, ly, q);
    S3[q] = SCHEME == 1 ? 0.0 : 0.5 * ((ns(PK, lx, ly) - 4.0 * pk) * ih2);
    if (phik_copy) phik_copy[q] = pk;
    phi0[q] = G0[ly][lx];
    ka[q] = K[ly][lx];
    mu[q] = MU[ly][lx];
    if constexpr (NORM) {
        const double lmu = (ns(MU, lx, ly) - 4.0 * MU[ly][lx]) * ih2;
        const double r1 = s1 - (G0[ly][lx] - op.c * lmu);
        const double bs = block_sum<NT>(r1 * r1, red);
        if (t == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = bs;
    }
}

// Residual norm of a guess completed by k_setup and k_complete_mu: N^(2) = S^(2)
// and N^(3) = S^(3) hold by construction (up to rounding), so only
// r1 = S1 - (phi - c Lap mu) is summed (per-block sums of r1^2 into part[];
// k_norm_finalize turns them into the norm).  Reads phi, mu and S1.
template <int NT>
__global__ void __launch_bounds__(NT) k_resnorm_guess(Fields<double> F, LevelOp<double> op, Grid g,
                                                      double* part) {
    __shared__ double red[NT / 64];
    double acc = 0.0;
    const size_t total = (size_t)g.m * g.n;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        int i, j;
        cell_of(q, g, i, j);
        const double lmu = (nsum(F.mu, i, j, g) - 4.0 * F.mu[q]) * op.ih2;
        const double r1 = F.f1[q] - (F.phi[q] - op.c * lmu);
        acc += r1 * r1;
    }
    const double bs = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

__global__ void __launch_bounds__(256) k_complete_kappa(Grid g, double ih2, double e,
                                                        const double* __restrict__ phi,
                                                        const double* __restrict__ S3,
                                                        double* ka) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.m || j >= g.n) return;
    complete_kappa_cell(g, ih2, e, phi, S3, ka, i, j);
}

// ... and mu = S2 + g(phi) + al phi + Lap kappa (so N^(2) = S^(2)); the
// cell's phi is x.
template <int SCHEME>
__device__ __forceinline__ void complete_mu_at(const Grid& g, double ih2, double al, double x,
                                               const double* __restrict__ phik,
                                               const double* __restrict__ ka,
                                               const double* __restrict__ S2, double* mu, int i,
                                               int j, const double* __restrict__ pin) {
    const size_t q = at(i, j, g);
    const double xk = SCHEME == 2 ? phik[q] : 0.0;
    const double alq = al + (pin ? pin[q] : 0.0);
    mu[q] = S2[q] + nl_value<double, SCHEME, false>(x, 0.0, xk) + alq * x +
            (nsum(ka, i, j, g) - 4.0 * ka[q]) * ih2;
}

template <int SCHEME>
__device__ __forceinline__ void complete_mu_cell(const Grid& g, double ih2, double al,
                                                 const double* __restrict__ phi,
                                                 const double* __restrict__ phik,
                                                 const double* __restrict__ ka,
                                                 const double* __restrict__ S2, double* mu, int i,
                                                 int j, const double* __restrict__ pin = nullptr) {
    complete_mu_at<SCHEME>(g, ih2, al, phi[at(i, j, g)], phik, ka, S2, mu, i, j, pin);
}

template <int SCHEME>
__global__ void __launch_bounds__(256) k_complete_mu(Grid g, double ih2, double al,
                                                     const double* __restrict__ phi,
                                                     const double* __restrict__ phik,
                                                     const double* __restrict__ ka,
                                                     const double* __restrict__ S2, double* mu,
                                                     const double* __restrict__ pin) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.m || j >= g.n) return;
    complete_mu_cell<SCHEME>(g, ih2, al, phi, phik, ka, S2, mu, i, j, pin);
}

// 2x2 average (restriction of phi^k for the scheme-2 coarse operators).
template <typename TI, typename TO>
__global__ void __launch_bounds__(256) k_restrict(Grid g, const TI* __restrict__ f, TO* fc) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int mc = g.m >> 1, nc = g.n >> 1;
    if (I >= mc || J >= nc) return;
    const TI s = (f[at(2 * I, 2 * J, g)] + f[at(2 * I + 1, 2 * J, g)]) +
                 (f[at(2 * I, 2 * J + 1, g)] + f[at(2 * I + 1, 2 * J + 1, g)]);
    fc[(size_t)J * mc + I] = (TO)(TI(0.25) * s);
}

// psi^{k+1}: (phi - phi^k)/s (scheme 1, eq. discrete_1_b) or
// (2/s)(phi - phi^k) - psi^k (scheme 2, eq. discrete_2_b); in place on psi.
// phi is also copied to phi_out (the caller's phi^{k+1}).
template <int SCHEME>
__device__ __forceinline__ void psi_cell(double s, const double* __restrict__ phi,
                                         const double* __restrict__ phik, double* psi,
                                         double* phi_out, size_t q) {
    const double x = phi[q];
    if constexpr (SCHEME == 1) psi[q] = (x - phik[q]) / s;
    else psi[q] = (2.0 / s) * (x - phik[q]) - psi[q];
    phi_out[q] = x;
}

template <int SCHEME>
__global__ void __launch_bounds__(256) k_psi_update(size_t total, double s,
                                                    const double* __restrict__ phi,
                                                    const double* __restrict__ phik, double* psi,
                                                    double* phi_out) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    psi_cell<SCHEME>(s, phi, phik, psi, phi_out, q);
}

}  // namespace mpfc
