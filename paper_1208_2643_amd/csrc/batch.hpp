// Batched kernels: many independent MPFC simulations (own grid size and
// parameters, same scheme) advanced together, one launch per phase of the
// time step instead of one per simulation.
//
// Every batched launch walks a work list of BatchItem {arg, tile}: `arg`
// selects the simulation's argument record in a device table, `tile` the
// piece of its grid this workgroup handles.  The cell kernels here take
// chunks of BCHUNK cells of the finest grid; the V-cycle tiles and the
// persistent coarse levels are the batched forms of the single-grid kernels
// (k_tile_batched, k_coarse_persistent_batched).  Each simulation keeps its
// own stop flag: once it has converged its items return at once, while the
// others go on.  The arithmetic of every cell is the single-grid one (the
// per-cell device functions of kernels.hpp), so a simulation's iterates do not
// depend on what it is batched with.
#pragma once
#include "step.hpp"
#include "tiles.hpp"

namespace mpfc {

constexpr int BCHUNK = 1024;  // cells per item of the cell kernels (256 threads x 4)

// Per-simulation record of the cell kernels.  Pointers are into the
// simulation's own device arena (finest level).
struct BSim {
    Grid g;
    double ih2, h2;
    double d, alpha;            // source: weight of psi^k, alpha = 1 - eps
    double al, e;               // N^(2) linear weight, N^(3) Laplacian weight
    double dt;
    LevelOp<double> op;
    double* S[3];               // source
    double* phik;               // copy of phi^k
    double* u[2][3];            // FP64 iterate copies (u[1] only with mixed precision)
    float* fe[3];               // FP32 correction (mixed)
    float* fr[3];               // FP32 residual (mixed)
    float* fpb;                 // FP32 base phi (mixed)
    float* fxk;                 // FP32 phi^k (mixed, scheme 2)
    CycleState* st;
    double* hist;
    double* part;               // per-item partial sums of r^2
    int nchunks;                // m n / BCHUNK: partials of the cell kernels
    int ntiles_up;              // partials of the finest up launch (its tile count)
};

// Caller's buffers of one step (rewritten before every step).
struct BIo {
    const double* phin;
    const double* phinm1;
    double* psi;
    double* phinp1;
};

// Cells of item `chunk`: q = chunk * BCHUNK + k * 256 + t, k < 4 (coalesced).
#define BATCH_CELLS(S, chunk, ...)                                                    \
    for (int k_ = 0; k_ < BCHUNK / 256; ++k_) {                                       \
        const size_t q = (size_t)(chunk) * BCHUNK + (size_t)k_ * 256 + threadIdx.x;   \
        const int i = (int)(q & (size_t)((S).g.m - 1));                               \
        const int j = (int)(q >> (S).g.lm);                                           \
        (void)i; (void)j;                                                             \
        __VA_ARGS__                                                                   \
    }

// Step set-up, part 1: source S, copy of phi^k, guess phi^(0).
template <int SCHEME>
__global__ void __launch_bounds__(256) k_b_setup(const BSim* __restrict__ sims,
                                                 const BIo* __restrict__ io,
                                                 const BatchItem* __restrict__ items, int mode) {
    const BatchItem it = items[blockIdx.x];
    const BSim& S = sims[it.arg];
    const BIo& O = io[it.arg];
    BATCH_CELLS(S, it.tile, {
        source_cell<SCHEME>(S.g, S.ih2, S.d, S.alpha, O.phin, O.phinm1, O.psi, S.S[0], S.S[1],
                            S.S[2], S.phik, i, j);
        S.u[0][0][q] = guess_value(mode, O.phin[q], O.phinm1[q]);
    })
}

// Part 2: kappa completion.
__global__ void __launch_bounds__(256) k_b_kappa(const BSim* __restrict__ sims,
                                                 const BatchItem* __restrict__ items) {
    const BatchItem it = items[blockIdx.x];
    const BSim& S = sims[it.arg];
    BATCH_CELLS(S, it.tile, {
        complete_kappa_cell(S.g, S.ih2, S.e, S.u[0][0], S.S[2], S.u[0][2], i, j);
    })
}

// Part 3: mu completion; with mixed precision (scheme 2) also phi^k in FP32.
template <int SCHEME, bool MIXED>
__global__ void __launch_bounds__(256) k_b_mu(const BSim* __restrict__ sims,
                                              const BatchItem* __restrict__ items) {
    const BatchItem it = items[blockIdx.x];
    const BSim& S = sims[it.arg];
    BATCH_CELLS(S, it.tile, {
        complete_mu_cell<SCHEME>(S.g, S.ih2, S.al, S.u[0][0], S.phik, S.u[0][2], S.S[1],
                                 S.u[0][1], i, j);
        if constexpr (MIXED && SCHEME == 2) S.fxk[q] = (float)S.phik[q];
    })
}

// Reset every simulation's cycle state.
__global__ void __launch_bounds__(64) k_b_state_reset(const BSim* __restrict__ sims, int nsim) {
    const int s = blockIdx.x * 64 + threadIdx.x;
    if (s >= nsim) return;
    CycleState* st = sims[s].st;
    st->acc = 0.0; st->blocks = 0u; st->count = 0;
    st->status = ST_RUNNING; st->done = 0; st->pad0 = st->pad1 = 0;
}

// FP64 residual of the iterate u[0]: per-item sum of r^2 into part[chunk].
template <int SCHEME>
__global__ void __launch_bounds__(256) k_b_resnorm(const BSim* __restrict__ sims,
                                                   const BatchItem* __restrict__ items) {
    const BatchItem it = items[blockIdx.x];
    const BSim& S = sims[it.arg];
    if (stopped(S.st)) return;
    __shared__ double red[4];
    Fields<double> F;
    F.phi = S.u[0][0]; F.mu = S.u[0][1]; F.ka = S.u[0][2];
    F.f1 = S.S[0]; F.f2 = S.S[1]; F.f3 = S.S[2];
    F.phik = S.phik; F.base = nullptr;
    double acc = 0.0;
    BATCH_CELLS(S, it.tile, {
        double a, b, c;
        residual_at<double, SCHEME, false>(F, S.op, S.g, i, j, a, b, c);
        acc += a * a + b * b + c * c;
    })
    const double bs = block_sum<256>(acc, red);
    if (threadIdx.x == 0) S.part[it.tile] = bs;
}

// Mixed precision: FP64 defect step u[from] (+ e) -> u[from ^ 1], FP32 residual
// and base phi, per-item sum of r^2.
template <int SCHEME>
__global__ void __launch_bounds__(256) k_b_defect(const BSim* __restrict__ sims,
                                                  const BatchItem* __restrict__ items, int from,
                                                  int add) {
    const BatchItem it = items[blockIdx.x];
    const BSim& S = sims[it.arg];
    if (stopped(S.st)) return;
    __shared__ double red[4];
    const int to = from ^ 1;
    Fields<double> F;
    F.phi = S.u[from][0]; F.mu = S.u[from][1]; F.ka = S.u[from][2];
    F.f1 = S.S[0]; F.f2 = S.S[1]; F.f3 = S.S[2];
    F.phik = S.phik; F.base = nullptr;
    double acc = 0.0;
    BATCH_CELLS(S, it.tile, {
        acc += defect_cell<SCHEME>(F, S.op, S.g, S.fe[0], S.fe[1], S.fe[2], add, S.u[to][0],
                                   S.u[to][1], S.u[to][2], S.fr[0], S.fr[1], S.fr[2], S.fpb, i, j);
    })
    const double bs = block_sum<256>(acc, red);
    if (threadIdx.x == 0) S.part[it.tile] = bs;
}

// Mixed precision: clear the FP32 correction before an outer iteration.
__global__ void __launch_bounds__(256) k_b_clear_e(const BSim* __restrict__ sims,
                                                   const BatchItem* __restrict__ items) {
    const BatchItem it = items[blockIdx.x];
    const BSim& S = sims[it.arg];
    if (stopped(S.st)) return;
    BATCH_CELLS(S, it.tile, {
        S.fe[0][q] = 0.f; S.fe[1][q] = 0.f; S.fe[2][q] = 0.f;
    })
}

// Norm, history and stop decision of every simulation: workgroup s sums
// simulation s's partials.
// `tiles` = 1: the partials come from the finest up launch, else from a cell kernel.
template <int NT>
__global__ void __launch_bounds__(NT) k_b_finalize(const BSim* __restrict__ sims, int tiles,
                                                   double tol, int max_norms, double diverge) {
    const BSim& S = sims[blockIdx.x];
    if (stopped(S.st)) return;
    norm_finalize_body<NT>(S.part, tiles ? S.ntiles_up : S.nchunks, S.st, S.hist, S.h2, tol,
                           max_norms, diverge);
}

// Wrap-up: psi update and copy-out from the FP64 copy that holds the solution
// (always u[0] in FP64; with mixed precision copy 1 ^ (outer iterations & 1),
// read from the simulation's own cycle count).
template <int SCHEME, bool MIXED>
__global__ void __launch_bounds__(256) k_b_psi(const BSim* __restrict__ sims,
                                               const BIo* __restrict__ io,
                                               const BatchItem* __restrict__ items) {
    const BatchItem it = items[blockIdx.x];
    const BSim& S = sims[it.arg];
    const BIo& O = io[it.arg];
    int cur = 0;
    if constexpr (MIXED) cur = 1 ^ ((S.st->count - 1) & 1);
    const double* phi = S.u[cur][0];
    BATCH_CELLS(S, it.tile, { psi_cell<SCHEME>(S.dt, phi, O.phin, O.psi, O.phinp1, q); })
}

#undef BATCH_CELLS

}  // namespace mpfc
