// Periodic Poisson multigrid and energy reductions (FP64), used for the
// discrete energies of the MPFC schemes (Sec. 3; App. A).
//
// The "-1" norm of a mean-zero grid function psi is ||psi||_{-1}^2 = h^2 (psi, w)
// with -Lap_h w = psi, w periodic and mean-zero (App. A, mean-zero space H).
// w is found by a linear multigrid V-cycle (red-black Gauss-Seidel, 2x2
// average restriction of the residual, bilinear prolongation of the
// correction, exact solve on the coarsest grid with a precomputed periodic
// Green's matrix).
#pragma once
#include "kernels.hpp"

namespace mpfc {

// The block-sum result of thread 0 is added to *dst with one atomic.
template <int NT>
__device__ __forceinline__ void block_atomic_add(double v, double* red, double* dst) {
    const double s = block_sum<NT>(v, red);
    if (threadIdx.x == 0) atomicAdd(dst, s);
    __syncthreads();
}

__global__ void k_zero(double* a, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = 0.0;
}

template <typename T>
__global__ void __launch_bounds__(256) k_fill(T* a, size_t n, T v) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = v;
}

template <typename T>
__global__ void __launch_bounds__(256) k_copy(T* dst, const T* __restrict__ src, size_t n) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) dst[t] = src[t];
}

// acc[0] += sum f
template <int NT>
__global__ void __launch_bounds__(NT) k_sum(const double* __restrict__ f, size_t total, double* acc) {
    __shared__ double red[NT / 64];
    double s = 0.0;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT)
        s += f[q];
    block_atomic_add<NT>(s, red, acc);
}

// b = psi - mean(psi) (mean = sum[0]/total); acc[0] += sum b^2.
template <int NT>
__global__ void __launch_bounds__(NT) k_p_rhs(const double* __restrict__ psi, size_t total,
                                              const double* __restrict__ sum, double* b,
                                              double* acc) {
    __shared__ double red[NT / 64];
    const double mean = sum[0] / (double)total;
    double s = 0.0;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        const double v = psi[q] - mean;
        b[q] = v;
        s += v * v;
    }
    block_atomic_add<NT>(s, red, acc);
}

// Advance the Poisson solution across a time step.  With -Lap_h w^k = psi^k,
// the scheme's psi equation (eq. scheme1_1 or mpfc_scheme2_1 with the psi
// update) gives -Lap_h w^{k+1} = psi^{k+1} for w^{k+1} = a w^k - b (mu - mean mu),
// a = 1/(1 + s beta), b = s M/(1 + s beta) (scheme 1) or a = (1 - s beta/2)/
// (1 + s beta/2), b = s M/(1 + s beta/2) (scheme 2), up to the step's residual.
__global__ void __launch_bounds__(256) k_w_advance(double* w, const double* __restrict__ mu,
                                                   size_t total, double a, double b,
                                                   const double* __restrict__ musum) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const double mean = musum[0] / (double)total;
    w[q] = a * w[q] - b * (mu[q] - mean);
}

// Finest-grid Poisson residual norm with the same last-block bookkeeping as
// the nonlinear solve; tolerance rtol * ||b|| (bnorm2 = sum b^2).
template <int NT>
__global__ void __launch_bounds__(NT) k_p_resnorm(const double* __restrict__ w,
                                                  const double* __restrict__ b, Grid g, double ih2,
                                                  CycleState* st, double* hist,
                                                  const double* __restrict__ bnorm2, double rtol,
                                                  int max_norms) {
    if (stopped(st)) return;
    __shared__ double red[NT / 64];
    __shared__ int last;
    double acc = 0.0;
    const size_t total = (size_t)g.m * g.n;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        const int i = (int)(q & (size_t)(g.m - 1));
        const int j = (int)(q >> g.lm);
        const double r = b[q] + (nsum(w, i, j, g) - 4.0 * w[q]) * ih2;
        acc += r * r;
    }
    const double bs = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) {
        atomicAdd(&st->acc, bs);
        __threadfence();
        const unsigned t = atomicAdd(&st->blocks, 1u);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        __threadfence();
        const double nr = sqrt(atomicAdd(&st->acc, 0.0));
        const int k = st->count;
        hist[k] = nr;
        st->count = k + 1;
        int status = ST_RUNNING;
        if (!(nr == nr)) status = ST_NONFINITE;
        else if (nr <= rtol * sqrt(bnorm2[0]) || nr == 0.0) status = ST_CONVERGED;
        else if (k + 1 >= max_norms) status = ST_MAXCYC;
        st->status = status;
        st->done = status != ST_RUNNING;
        st->acc = 0.0;
        st->blocks = 0u;
        __threadfence();
    }
}

// Energy sums after a step (Sec. 3, eqs. discrete_energy_PFC, energy_numer;
// App. A norms):
//   acc[0] += sum phi^4, acc[1] += sum phi^2,
//   acc[2] += sum over east/north edges of (phi difference)^2,
//   acc[3] += sum (Lap_h phi)^2, acc[4] += sum phi,
//   acc[5] += sum over edges of (difference of phi - phi_prev)^2,
//   acc[6] += sum (psi - mean psi) w.
template <int NT>
__global__ void __launch_bounds__(NT) k_energy_terms(Grid g, double ih2,
                                                     const double* __restrict__ phi,
                                                     const double* __restrict__ phiprev,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ w, double* acc) {
    __shared__ double red[NT / 64];
    double a[7] = {0, 0, 0, 0, 0, 0, 0};
    const size_t total = (size_t)g.m * g.n;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        const int i = (int)(q & (size_t)(g.m - 1));
        const int j = (int)(q >> g.lm);
        const double x = phi[q];
        const double xe = phi[at(wrapx(i + 1, g), j, g)], xn = phi[at(i, wrapy(j + 1, g), g)];
        const double L = (nsum(phi, i, j, g) - 4.0 * x) * ih2;
        a[0] += (x * x) * (x * x);
        a[1] += x * x;
        a[2] += (xe - x) * (xe - x) + (xn - x) * (xn - x);
        a[3] += L * L;
        a[4] += x;
        if (phiprev) {
            const double d = x - phiprev[q];
            const double de = xe - phiprev[at(wrapx(i + 1, g), j, g)] - d;
            const double dn = xn - phiprev[at(i, wrapy(j + 1, g), g)] - d;
            a[5] += de * de + dn * dn;
        }
        a[6] += b[q] * w[q];
    }
#pragma unroll
    for (int k = 0; k < 7; ++k) block_atomic_add<NT>(a[k], red, acc + k);
}

}  // namespace mpfc
