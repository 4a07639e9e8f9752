// Reductions and helpers for the discrete energies of the MPFC schemes
// (Sec. 3; App. A).
//
// The "-1" norm of a mean-zero grid function psi is ||psi||_{-1}^2 = h^2 (psi, w)
// with -Lap_h w = psi, w mean-zero with the grid's boundary conditions (App. A,
// mean-zero space H).
// w is found with the same V-cycle kernels as the MPFC system (tiles.hpp,
// PoissonOp): red-black Gauss-Seidel, 2x2-average restriction, bilinear
// prolongation, and on the coarsest grid a precomputed Green's matrix.
//
// Every reduction writes one partial sum per block (no atomics, no
// device-wide fences); k_partials_sum adds them in a fixed order, so all sums
// are deterministic.
#pragma once
#include "step.hpp"

namespace mpfc {

template <typename T>
__global__ void __launch_bounds__(256) k_fill(T* a, size_t n, T v) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = v;
}

// out[k] = sum over b < nparts of part[b * nvals + k], for k < nvals <= NT (one
// block).  Thread t < (NT / nvals) * nvals adds the values of one k in a
// fixed stride, reading consecutive addresses with its neighbours; then
// thread k adds the NT / nvals thread sums of value k in order.
template <int NT>
__device__ __forceinline__ double partials_sum_body(const double* __restrict__ part, int nparts,
                                                    int nvals, double* out) {
    __shared__ double red[NT];
    const int t = threadIdx.x, per = NT / nvals;
    double s = 0.0;
    if (t < per * nvals) {
        // four loads in flight per thread: blocks b, b + per, b + 2 per, b + 3 per
        const int k = t % nvals;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int b = t / nvals;
        for (; b + 3 * per < nparts; b += 4 * per) {
            s0 += part[(size_t)b * nvals + k];
            s1 += part[(size_t)(b + per) * nvals + k];
            s2 += part[(size_t)(b + 2 * per) * nvals + k];
            s3 += part[(size_t)(b + 3 * per) * nvals + k];
        }
        for (; b < nparts; b += per) s0 += part[(size_t)b * nvals + k];
        s = (s0 + s1) + (s2 + s3);
    }
    red[t] = s;
    __syncthreads();
    double tot = 0.0;
    if (t < nvals) {
        for (int r = 0; r < per; ++r) tot += red[r * nvals + t];
        out[t] = tot;
    }
    return tot;  // value t for threads t < nvals
}

template <int NT>
__global__ void __launch_bounds__(NT) k_partials_sum(const double* __restrict__ part, int nparts,
                                                     int nvals, double* out) {
    partials_sum_body<NT>(part, nparts, nvals, out);
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

// Norm bookkeeping of the Poisson cycles and the stop decision for one norm
// (one thread): `tot` the squared residual sum, `bsq` = ||b||^2.
__device__ inline void p_decide(CycleState* st, double* hist, double tot, double bsq, double rel,
                                double stall, int max_norms) {
    const double nr = sqrt(tot);
    const double bn = sqrt(bsq);
    const int k = st->count;
    const double prev = k > 0 ? hist[k - 1] : 1e300;
    hist[k] = nr;
    st->acc = nr;
    st->count = k + 1;
    int status = ST_RUNNING;
    if (!(nr == nr)) status = ST_NONFINITE;
    else if (bn == 0.0 || nr <= rel * bn || (nr <= stall * bn && nr > 0.5 * prev))
        status = ST_CONVERGED;
    else if (k + 1 >= max_norms) status = ST_MAXCYC;
    st->status = status;
    st->done = status != ST_RUNNING;
}

// Norm bookkeeping of the Poisson cycles with the stop decision on the device:
// converged when ||r|| <= rel ||b|| (||b||^2 = bsq[0]), or when the residual has
// reached the operator's rounding floor (||r|| <= stall ||b|| and the last cycle
// removed less than half of it), or b = 0; the cycle limit gives ST_MAXCYC.
template <int NT>
__global__ void __launch_bounds__(NT) k_p_finalize(const double* __restrict__ part, int nparts,
                                                   CycleState* st, double* hist,
                                                   const double* __restrict__ bsq, double rel,
                                                   double stall, int max_norms) {
    if (stopped(st)) return;
    __shared__ double red[NT / 64];
    double s = 0.0;
    for (int b = threadIdx.x; b < nparts; b += NT) s += part[b];
    const double tot = block_sum<NT>(s, red);
    if (threadIdx.x == 0) p_decide(st, hist, tot, bsq[0], rel, stall, max_norms);
}

// Finest-grid Poisson residual sum of squares (b + Lap_h w)^2 for grids small
// enough that every level runs in the persistent kernel.
template <int NT>
__global__ void __launch_bounds__(NT) k_p_resnorm(const double* __restrict__ w,
                                                  const double* __restrict__ b, Grid g, double ih2,
                                                  const CycleState* st, double* part) {
    if (stopped(st)) return;
    __shared__ double red[NT / 64];
    double acc = 0.0;
    const size_t total = (size_t)g.m * g.n;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        int i, j;
        cell_of(q, g, i, j);
        const double r = b[q] + (nsum(w, i, j, g) - 4.0 * w[q]) * ih2;
        acc += r * r;
    }
    const double bs = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

// Step 1 of the energies: per-block sums of x and y (y may be null: 0) into
// part[blk * 2 + 0/1]; block 0 also resets the Poisson cycle state `st`.
template <int NT>
__global__ void __launch_bounds__(NT) k_sum2(const double* __restrict__ x,
                                             const double* __restrict__ y, size_t total,
                                             double* part, CycleState* st) {
    __shared__ double red[NT / 64];
    if (st && blockIdx.x == 0 && threadIdx.x == 0) {
        st->acc = 0.0; st->blocks = 0u; st->count = 0;
        st->status = ST_RUNNING; st->done = 0; st->pad0 = st->pad1 = 0;
    }
    double sx = 0.0, sy = 0.0;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        sx += x[q];
        if (y) sy += y[q];
    }
    const double tx = block_sum<NT>(sx, red);
    __syncthreads();
    const double ty = block_sum<NT>(sy, red);
    if (threadIdx.x == 0) {
        part[(size_t)blockIdx.x * 2] = tx;
        part[(size_t)blockIdx.x * 2 + 1] = ty;
    }
}

// b = psi - mean(psi) (mean = sum[0] / total) and per-block sums of b^2 and,
// when w is given, of r^2 with r = b - (-Lap_h w), the residual of the warm
// start before any cycle, into part[blk * 2 + 0/1].
template <int NT>
__device__ __forceinline__ void p_rhs_resid_body(Grid g, double ih2,
                                                 const double* __restrict__ psi,
                                                 const double* __restrict__ sum, double* b,
                                                 const double* __restrict__ w, double* part) {
    __shared__ double red[NT / 64];
    const size_t total = (size_t)g.m * g.n;
    const double mean = sum[0] / (double)total;
    double sb = 0.0, sr = 0.0;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        const double v = psi[q] - mean;
        b[q] = v;
        sb += v * v;
        if (w) {
            int i, j;
            cell_of(q, g, i, j);
            const double r = v - (4.0 * w[q] - nsum(w, i, j, g)) * ih2;
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

template <int NT>
__global__ void __launch_bounds__(NT) k_p_rhs_resid(Grid g, double ih2,
                                                    const double* __restrict__ psi,
                                                    const double* __restrict__ sum, double* b,
                                                    const double* __restrict__ w, double* part) {
    p_rhs_resid_body<NT>(g, ih2, psi, sum, b, w, part);
}

// Energy sums after a step (Sec. 3, eqs. discrete_energy_PFC, energy_numer;
// App. A norms), per block into part[blk * 8 + k]:
//   k = 0: sum phi^4, 1: sum phi^2,
//   2: sum over east/north edges of (phi difference)^2,
//   3: sum (Lap_h phi)^2, 4: sum phi,
//   5: sum over edges of (difference of phi - phi_prev)^2,
//   6: sum (psi - mean psi) w,
//   7: sum W (phi - phi_hat)^2 (pinning, Sec. 4.6; 0 without pinning).
template <int NT>
__device__ __forceinline__ void energy_terms_body(Grid g, double ih2,
                                                  const double* __restrict__ phi,
                                                  const double* __restrict__ phiprev,
                                                  const double* __restrict__ b,
                                                  const double* __restrict__ w, double* part,
                                                  const double* __restrict__ pin,
                                                  const double* __restrict__ phihat) {
    __shared__ double red[NT / 64];
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const size_t total = (size_t)g.m * g.n;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        int i, j;
        cell_of(q, g, i, j);
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
        if (pin) {  // pinning energy sum W (phi - phi_hat)^2 (Sec. 4.6)
            const double dp = x - phihat[q];
            a[7] += pin[q] * dp * dp;
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double tot = block_sum<NT>(a[k], red);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * 8 + k] = tot;
        __syncthreads();
    }
}

template <int NT>
__global__ void __launch_bounds__(NT) k_energy_terms(Grid g, double ih2,
                                                     const double* __restrict__ phi,
                                                     const double* __restrict__ phiprev,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ w, double* part,
                                                     const double* __restrict__ pin,
                                                     const double* __restrict__ phihat) {
    energy_terms_body<NT>(g, ih2, phi, phiprev, b, w, part, pin, phihat);
}

}  // namespace mpfc
