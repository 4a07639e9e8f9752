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

// psi^{k+1} in place on the caller's psi and phi^{k+1} into the caller's array.
template <int SCHEME>
__global__ void __launch_bounds__(256) k_wrap_psi(const StepIO* __restrict__ io,
                                                  const CycleState* st, int mixed,
                                                  const double* __restrict__ phi0,
                                                  const double* __restrict__ phi1, size_t total,
                                                  double s) {
    if (wrapup_off(st)) return;
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const double* phi = final_copy(st, mixed) ? phi1 : phi0;
    psi_cell<SCHEME>(s, phi, io->phi_n, io->psi, io->phi_np1, q);
}

// Per-block sums of psi^{k+1} and (advance) of the step's mu into
// part[blk * 2 + 0/1]; block 0 resets the Poisson cycle state, or, while the
// wrap-up is off, marks it stopped so that the Poisson cycles skip too.
template <int NT>
__global__ void __launch_bounds__(NT) k_wrap_sums(const StepIO* __restrict__ io,
                                                  const CycleState* st, int mixed,
                                                  const double* __restrict__ mu0,
                                                  const double* __restrict__ mu1, int advance,
                                                  size_t total, double* part, CycleState* pst) {
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
    const double* x = io->psi;
    const double* y = advance ? (final_copy(st, mixed) ? mu1 : mu0) : nullptr;
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

template <int NT>
__global__ void __launch_bounds__(NT) k_wrap_partials(const CycleState* st,
                                                      const double* __restrict__ part, int nparts,
                                                      int nvals, double* out) {
    if (wrapup_off(st)) return;
    partials_sum_body<NT>(part, nparts, nvals, out);
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

// b = psi^{k+1} - mean and the sums of b^2 and of the warm start's residual.
template <int NT>
__global__ void __launch_bounds__(NT) k_wrap_rhs_resid(const CycleState* st,
                                                       const StepIO* __restrict__ io, Grid g,
                                                       double ih2, const double* __restrict__ sum,
                                                       double* b, const double* __restrict__ w,
                                                       double* part) {
    if (wrapup_off(st)) return;
    p_rhs_resid_body<NT>(g, ih2, io->psi, sum, b, w, part);
}

// Energy sums of phi^{k+1} (the caller's array, written by k_wrap_psi) with
// phi^k as the previous state.
template <int NT>
__global__ void __launch_bounds__(NT) k_wrap_terms(const CycleState* st,
                                                   const StepIO* __restrict__ io, Grid g,
                                                   double ih2, const double* __restrict__ b,
                                                   const double* __restrict__ w, double* part,
                                                   const double* __restrict__ pin,
                                                   const double* __restrict__ phihat) {
    if (wrapup_off(st)) return;
    energy_terms_body<NT>(g, ih2, io->phi_np1, io->phi_n, b, w, part, pin, phihat);
}

}  // namespace mpfc
