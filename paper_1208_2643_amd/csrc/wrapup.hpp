// Kernels of the captured set-up and wrap-up of one time step.
//
// A step's set-up (source, guess, completion, first norm) and wrap-up (psi
// update, eqs. discrete_1_b / discrete_2_b, and the energies of Sec. 3) are
// replayed from captured graphs.  The caller's arrays change from step to
// step, so those kernels read them from a small device table (StepIO) that a
// one-thread kernel fills before the step.
//
// The wrap-up is enqueued right behind the predicted number of V-cycles,
// before the host knows whether they were enough: each of its kernels first
// checks the step's cycle state and does nothing unless the cycles have
// stopped (the Poisson cycles of the -1 norm are switched off through their
// own state).  When more cycles were needed the host runs them and then the
// wrap-up again.
#pragma once
#include "poisson.hpp"

namespace mpfc {

// The step's cycles have not stopped yet: the wrap-up waits for the host.
__device__ __forceinline__ bool wrapup_off(const CycleState* st) { return st->done == 0; }

// FP64 copy of the level-0 iterate that holds the result: copy 0, or with
// mixed precision copy 1 ^ (outer iterations & 1) (the outer iterations
// alternate between the two copies; count - 1 of them ran).
__device__ __forceinline__ int final_copy(const CycleState* st, int mixed) {
    return mixed ? 1 ^ ((st->count - 1) & 1) : 0;
}

// Level-0 arrays of the two FP64 copies of the iterate (copy 1 exists with
// mixed precision and with the learned guess; null otherwise).
struct WrapFields {
    const double* phi[2];
    const double* mu[2];
    const double* kappa[2];
};

// The caller's optional mu and kappa outputs of cell q from the final copy c.
__device__ __forceinline__ void wrap_outputs(const StepIO* __restrict__ io, const WrapFields& f,
                                             int c, size_t q) {
    if (io->mu) io->mu[q] = f.mu[c][q];
    if (io->kappa) io->kappa[q] = f.kappa[c][q];
}

// psi^{k+1} in place on the caller's psi, phi^{k+1} and (when asked for) mu,
// kappa into the caller's arrays (steps without energies).
template <int SCHEME>
__global__ void __launch_bounds__(256) k_wrap_psi(const StepIO* __restrict__ io,
                                                  const CycleState* st, int mixed, WrapFields f,
                                                  size_t total, double s) {
    if (wrapup_off(st)) return;
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int c = final_copy(st, mixed);
    psi_cell<SCHEME>(s, f.phi[c], io->phi_n, io->psi, io->phi_np1, q);
    wrap_outputs(io, f, c, q);
}

// psi^{k+1} in place on the caller's psi, phi^{k+1} and (when asked for) mu,
// kappa into the caller's arrays, and per-block sums of psi^{k+1} and
// (advance) of the step's mu into part[blk * 2 + 0/1].  Block 0 resets the
// Poisson cycle state, or, while the wrap-up is off, marks it stopped so that
// the Poisson cycles skip too.
template <int SCHEME, int NT>
__global__ void __launch_bounds__(NT) k_wrap_psi_sums(const StepIO* __restrict__ io,
                                                      const CycleState* st, int mixed,
                                                      WrapFields f, int advance, size_t total,
                                                      double s, double* part, CycleState* pst) {
    __shared__ double red[NT / 64];
    const bool off = wrapup_off(st);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (off) {
            pst->done = 1;
        } else {
            pst->acc = 0.0; pst->blocks = 0u; pst->count = 0;
            pst->status = ST_RUNNING; pst->done = 0; pst->pad0 = pst->pad1 = 0;
        }
    }
    if (off) return;
    const int fc = final_copy(st, mixed);
    const double* __restrict__ phi = f.phi[fc];
    const double* __restrict__ mu = f.mu[fc];
    const double* __restrict__ ka = f.kappa[fc];
    const double* __restrict__ phik = io->phi_n;
    double* __restrict__ psi = io->psi;
    double* __restrict__ out = io->phi_np1;
    double* __restrict__ mu_out = io->mu;
    double* __restrict__ ka_out = io->kappa;
    double sx = 0.0, sy = 0.0;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        const double x = phi[q];
        const double v = SCHEME == 1 ? (x - phik[q]) / s : (2.0 / s) * (x - phik[q]) - psi[q];
        psi[q] = v;
        out[q] = x;
        sx += v;
        if (advance || mu_out) {
            const double y = mu[q];
            if (advance) sy += y;
            if (mu_out) mu_out[q] = y;
        }
        if (ka_out) ka_out[q] = ka[q];
    }
    const double tx = block_sum<NT>(sx, red);
    __syncthreads();
    const double ty = block_sum<NT>(sy, red);
    if (threadIdx.x == 0) {
        part[(size_t)blockIdx.x * 2] = tx;
        part[(size_t)blockIdx.x * 2 + 1] = ty;
    }
}

template <int NT>
__global__ void __launch_bounds__(NT) k_wrap_partials(const CycleState* st,
                                                      const double* __restrict__ part, int nparts,
                                                      int nvals, double* out) {
    if (wrapup_off(st)) return;
    partials_sum_body<NT>(part, nparts, nvals, out);
}

// k_wrap_partials for the twelve sums of k_wrap_rhs_terms followed, for a
// warm start, by the Poisson state's first norm and stop decision from the
// warm start's residual sum (value 11) and ||b||^2 (value 10), as
// k_p_finalize would take them from acc[11] and acc[10].
template <int NT>
__global__ void __launch_bounds__(NT) k_wrap_partials_pnorm(const CycleState* st,
                                                            const double* __restrict__ part,
                                                            int nparts, double* out,
                                                            CycleState* pst, double* phist,
                                                            double rel, double stall,
                                                            int max_norms) {
    if (wrapup_off(st)) return;
    __shared__ double r[2];
    const double v = partials_sum_body<NT>(part, nparts, 12, out);
    if (threadIdx.x == 10) r[0] = v;
    if (threadIdx.x == 11) r[1] = v;
    __syncthreads();
    if (threadIdx.x == 0 && !stopped(pst)) p_decide(pst, phist, r[1], r[0], rel, stall, max_norms);
}

// Cold start of the Poisson solution (first step of a context).
__global__ void __launch_bounds__(256) k_wrap_w_zero(const CycleState* st, double* w,
                                                     size_t total) {
    if (wrapup_off(st)) return;
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < total) w[q] = 0.0;
}

// Warm start w^{k+1} = a w^k - b (mu - mean mu) (see k_w_advance).
__global__ void __launch_bounds__(256) k_wrap_w_advance(const CycleState* st, int mixed,
                                                        const double* __restrict__ mu0,
                                                        const double* __restrict__ mu1, double* w,
                                                        size_t total, double a, double b,
                                                        const double* __restrict__ musum) {
    if (wrapup_off(st)) return;
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const double* mu = final_copy(st, mixed) ? mu1 : mu0;
    const double mean = musum[0] / (double)total;
    w[q] = a * w[q] - b * (mu[q] - mean);
}

// One pass over the grid after the psi update: b = psi^{k+1} - mean (the
// Poisson right-hand side), the sums of b^2 and of the warm start's squared
// residual (b + Lap_h w)^2 (w null: cold start, no residual), and the energy
// sums of phi^{k+1} with phi^k as the previous state (energy_terms_body's
// eight), per block into part[blk * 12 + k]: k < 8 the energy sums, 8 and 9
// zero, 10 the sum of b^2, 11 the residual sum (the slots of the step's
// accumulator array that the Poisson cycles read).  The term sum (b, w) uses
// the warm start; k_wrap_terms recomputes the energy sums when Poisson cycles
// ran.
template <int NT>
__global__ void __launch_bounds__(NT) k_wrap_rhs_terms(const CycleState* st,
                                                       const StepIO* __restrict__ io, Grid g,
                                                       double ih2,
                                                       const double* __restrict__ sum, double* b,
                                                       const double* __restrict__ w, double* part,
                                                       const double* __restrict__ pin,
                                                       const double* __restrict__ phihat) {
    if (wrapup_off(st)) return;
    __shared__ double red[NT / 64][10];
    const size_t total = (size_t)g.m * g.n;
    const double mean = sum[0] / (double)total;
    const double* __restrict__ phi = io->phi_np1;
    const double* __restrict__ phiprev = io->phi_n;
    const double* __restrict__ psi = io->psi;
    double* __restrict__ bo = b;
    double a[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    // two of a thread's cells per iteration, in the same order, so that the
    // loads of both are in flight together (four: 182 VGPRs, half the waves)
    auto cell = [&](size_t q) __attribute__((always_inline)) {
        int i, j;
        cell_of(q, g, i, j);
        const double v = psi[q] - mean;
        bo[q] = v;
        a[8] += v * v;
        if (w) {
            const double r = v - (4.0 * w[q] - nsum(w, i, j, g)) * ih2;
            a[9] += r * r;
            a[6] += v * w[q];
        }
        const double x = phi[q];
        const size_t qe = at(wrapx(i + 1, g), j, g), qn = at(i, wrapy(j + 1, g), g);
        const double xe = phi[qe], xn = phi[qn];
        const double L = (nsum(phi, i, j, g) - 4.0 * x) * ih2;
        a[0] += (x * x) * (x * x);
        a[1] += x * x;
        a[2] += (xe - x) * (xe - x) + (xn - x) * (xn - x);
        a[3] += L * L;
        a[4] += x;
        const double d = x - phiprev[q];
        const double de = xe - phiprev[qe] - d;
        const double dn = xn - phiprev[qn] - d;
        a[5] += de * de + dn * dn;
        if (pin) {  // pinning energy sum W (phi - phi_hat)^2 (Sec. 4.6)
            const double dp = x - phihat[q];
            a[7] += pin[q] * dp * dp;
        }
    };
    const size_t stride = (size_t)gridDim.x * NT;
    size_t q = (size_t)blockIdx.x * NT + threadIdx.x;
    for (; q + stride < total; q += 2 * stride) {
        cell(q);
        cell(q + stride);
    }
    for (; q < total; q += stride) cell(q);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        const double v = wave_sum(a[k]);
        if (lane == 0) red[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
        const int k = threadIdx.x < 8 ? threadIdx.x : threadIdx.x - 2;
        double s = 0.0;
        if (threadIdx.x < 8 || threadIdx.x >= 10) {
#pragma unroll
            for (int wv = 0; wv < NT / 64; ++wv) s += red[wv][k];
        }
        part[(size_t)blockIdx.x * 12 + threadIdx.x] = s;
    }
}

// The energy sums once more, with the solution w of the Poisson cycles, when
// any ran (cold start, or a warm start that did not pass the test); else the
// sums of k_wrap_rhs_terms stand.
__device__ __forceinline__ bool terms_again(const CycleState* st, const CycleState* pst,
                                            int warm) {
    return !wrapup_off(st) && (!warm || pst->count > 1);
}

template <int NT>
__global__ void __launch_bounds__(NT) k_wrap_terms(const CycleState* st, const CycleState* pst,
                                                   int warm, const StepIO* __restrict__ io,
                                                   Grid g, double ih2,
                                                   const double* __restrict__ b,
                                                   const double* __restrict__ w, double* part,
                                                   const double* __restrict__ pin,
                                                   const double* __restrict__ phihat) {
    if (!terms_again(st, pst, warm)) return;
    energy_terms_body<NT>(g, ih2, io->phi_np1, io->phi_n, b, w, part, pin, phihat);
}

template <int NT>
__global__ void __launch_bounds__(NT) k_wrap_terms_sum(const CycleState* st,
                                                       const CycleState* pst, int warm,
                                                       const double* __restrict__ part,
                                                       int nparts, double* out) {
    if (!terms_again(st, pst, warm)) return;
    partials_sum_body<NT>(part, nparts, 8, out);
}

}  // namespace mpfc
