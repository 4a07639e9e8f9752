// Definitions and explicit instantiations of the launchers declared in
// launch.hpp.  The build compiles this file once per operator group
// (-DMPFC_GROUP=0..7) in parallel; without MPFC_GROUP every group is built.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace mpfc {
namespace {

bool general_index(const Grid& g) { return g.lm < 0 || g.ln < 0; }

#ifndef MPFC_TILE_EXACT
#define MPFC_TILE_EXACT 1
#endif

template <class Op, bool UP, bool NEU, int K>
void tile_k(const Op& op, const TileArgs<typename Op::real>& A, const CycleState* stop,
            hipStream_t s, bool gen) {
    constexpr TileShape S = kShapes[K];
    const dim3 grid(A.g.m / A.tx, A.g.n / A.ty), blk(kTileThreads);
    if constexpr (std::is_same<typename Op::real, double>::value && gen_shape(K)) {
        if (gen) {
            hipLaunchKernelGGL((k_tile<Op, S.tx, S.ty, S.hmax, UP, NEU, true>), grid, blk, 0, s, op,
                               A, stop);
            return;
        }
    }
    // the shape's own tile and halo (the larger levels): compile-time extents
    if (MPFC_TILE_EXACT && A.tx == S.tx && A.ty == S.ty && A.H == S.hmax) {
        hipLaunchKernelGGL((k_tile<Op, S.tx, S.ty, S.hmax, UP, NEU, false, true>), grid, blk, 0, s,
                           op, A, stop);
        return;
    }
    hipLaunchKernelGGL((k_tile<Op, S.tx, S.ty, S.hmax, UP, NEU>), grid, blk, 0, s, op, A, stop);
}

template <class Op, bool UP, bool NEU>
void tile_bc(const Op& op, const TileArgs<typename Op::real>& A, int shape,
             const CycleState* stop, hipStream_t s) {
    const bool gen = general_index(A.g);
    if (gen) shape = shape == 2 ? 2 : 0;  // general-index kernels: shapes 0 and 2
    switch (shape) {
        case 0: tile_k<Op, UP, NEU, 0>(op, A, stop, s, gen); break;
        case 1: tile_k<Op, UP, NEU, 1>(op, A, stop, s, gen); break;
        case 2: tile_k<Op, UP, NEU, 2>(op, A, stop, s, gen); break;
        case 3: tile_k<Op, UP, NEU, 3>(op, A, stop, s, gen); break;
        case 4: tile_k<Op, UP, NEU, 4>(op, A, stop, s, gen); break;
        case 5: tile_k<Op, UP, NEU, 5>(op, A, stop, s, gen); break;
        default: tile_k<Op, UP, NEU, 6>(op, A, stop, s, gen); break;
    }
}

template <class Op, bool UP, bool NEU, int K>
void tile_batched_k(const BatchTile<Op>* args, const BatchItem* items, int n, hipStream_t s) {
    constexpr TileShape S = kShapes[K];
    hipLaunchKernelGGL((k_tile_batched<Op, S.tx, S.ty, S.hmax, UP, NEU>), dim3(n), dim3(kTileThreads), 0, s,
                       args, items, n);
}

template <class Op, bool UP, bool NEU>
void tile_batched_bc(int shape, const BatchTile<Op>* args, const BatchItem* items, int n,
                     hipStream_t s) {
    switch (shape) {
        case 0: tile_batched_k<Op, UP, NEU, 0>(args, items, n, s); break;
        case 1: tile_batched_k<Op, UP, NEU, 1>(args, items, n, s); break;
        case 2: tile_batched_k<Op, UP, NEU, 2>(args, items, n, s); break;
        case 3: tile_batched_k<Op, UP, NEU, 3>(args, items, n, s); break;
        case 4: tile_batched_k<Op, UP, NEU, 4>(args, items, n, s); break;
        case 5: tile_batched_k<Op, UP, NEU, 5>(args, items, n, s); break;
        default: tile_batched_k<Op, UP, NEU, 6>(args, items, n, s); break;
    }
}

}  // namespace

// Periodic grids run the instantiation without the Neumann ghost handling.
template <class Op, bool UP>
void launch_tile(const Op& op, const TileArgs<typename Op::real>& A, int shape,
                 const CycleState* stop, hipStream_t s) {
    if (A.g.bc) tile_bc<Op, UP, true>(op, A, shape, stop, s);
    else tile_bc<Op, UP, false>(op, A, shape, stop, s);
}

template <class Op>
void launch_coarse(const Op& op, const CoarseArgs<typename Op::real>& A, bool four,
                   const CycleState* stop, hipStream_t s) {
    const dim3 g1(1), blk(CP_THREADS);
    if (A.geo.bc) {
        if (four) hipLaunchKernelGGL((k_coarse_persistent<Op, CP_THREADS, 4, true>), g1, blk, 0, s, op, A, stop);
        else hipLaunchKernelGGL((k_coarse_persistent<Op, CP_THREADS, 8, true>), g1, blk, 0, s, op, A, stop);
    } else {
        if (four) hipLaunchKernelGGL((k_coarse_persistent<Op, CP_THREADS, 4, false>), g1, blk, 0, s, op, A, stop);
        else hipLaunchKernelGGL((k_coarse_persistent<Op, CP_THREADS, 8, false>), g1, blk, 0, s, op, A, stop);
    }
}

template <class Op>
void launch_coarsest_gen(const Op& op, const CoarseArgs<typename Op::real>& A,
                         const CycleState* stop, hipStream_t s) {
    const dim3 g1(1), blk(CG_THREADS);
    if (A.geo.bc) hipLaunchKernelGGL((k_coarsest_sweeps<Op, true>), g1, blk, 0, s, op, A, stop);
    else hipLaunchKernelGGL((k_coarsest_sweeps<Op, false>), g1, blk, 0, s, op, A, stop);
}

template <class Op, bool UP>
void launch_tile_batched(bool neu, int shape, const BatchTile<Op>* args, const BatchItem* items,
                         int n, hipStream_t s) {
    if (neu) tile_batched_bc<Op, UP, true>(shape, args, items, n, s);
    else tile_batched_bc<Op, UP, false>(shape, args, items, n, s);
}

template <class Op, int NC>
void launch_coarse_batched(bool neu, int nsim, const BatchCoarse<Op>* args, hipStream_t s) {
    if (neu) hipLaunchKernelGGL((k_coarse_persistent_batched<Op, CP_THREADS, NC, true>), dim3(nsim),
                                dim3(CP_THREADS), 0, s, args);
    else hipLaunchKernelGGL((k_coarse_persistent_batched<Op, CP_THREADS, NC, false>), dim3(nsim),
                            dim3(CP_THREADS), 0, s, args);
}

#define MPFC_INST_TILE(OP)                                                                   \
    template void launch_tile<OP, false>(const OP&, const TileArgs<OP::real>&, int,          \
                                         const CycleState*, hipStream_t);                    \
    template void launch_tile<OP, true>(const OP&, const TileArgs<OP::real>&, int,           \
                                        const CycleState*, hipStream_t);                     \
    template void launch_coarse<OP>(const OP&, const CoarseArgs<OP::real>&, bool,            \
                                    const CycleState*, hipStream_t);
#define MPFC_INST_GEN(OP)                                                                    \
    template void launch_coarsest_gen<OP>(const OP&, const CoarseArgs<OP::real>&,            \
                                          const CycleState*, hipStream_t);
#define MPFC_INST_BATCH(OP)                                                                  \
    template void launch_tile_batched<OP, false>(bool, int, const BatchTile<OP>*,            \
                                                 const BatchItem*, int, hipStream_t);        \
    template void launch_tile_batched<OP, true>(bool, int, const BatchTile<OP>*,             \
                                                const BatchItem*, int, hipStream_t);         \
    template void launch_coarse_batched<OP, 4>(bool, int, const BatchCoarse<OP>*, hipStream_t); \
    template void launch_coarse_batched<OP, 8>(bool, int, const BatchCoarse<OP>*, hipStream_t);

// Operator groups (one compilation each): the FP64 operators by scheme and
// linearisation (with the general-index coarsest level and the batched
// forms), the pinned operator, the FP32 correction operators of mixed
// precision (with the batched forms), and the Poisson operator of the -1 norm.
using S2N = MpfcOp<double, 2, true, false>;
using S2P = MpfcOp<double, 2, false, false>;
using S1N = MpfcOp<double, 1, true, false>;
using S1P = MpfcOp<double, 1, false, false>;
using S2Pin = MpfcOp<double, 2, true, false, true>;
using F2N = MpfcOp<float, 2, true, true>;
using F2P = MpfcOp<float, 2, false, true>;
using F1N = MpfcOp<float, 1, true, true>;
using F1P = MpfcOp<float, 1, false, true>;
using Poi = PoissonOp<double>;

#if !defined(MPFC_GROUP) || MPFC_GROUP == 0
MPFC_INST_TILE(S2N)
MPFC_INST_GEN(S2N)
MPFC_INST_BATCH(S2N)
#endif
#if !defined(MPFC_GROUP) || MPFC_GROUP == 1
MPFC_INST_TILE(S2P)
MPFC_INST_GEN(S2P)
MPFC_INST_BATCH(S2P)
#endif
#if !defined(MPFC_GROUP) || MPFC_GROUP == 2
MPFC_INST_TILE(S1N)
MPFC_INST_GEN(S1N)
MPFC_INST_BATCH(S1N)
#endif
#if !defined(MPFC_GROUP) || MPFC_GROUP == 3
MPFC_INST_TILE(S1P)
MPFC_INST_GEN(S1P)
MPFC_INST_BATCH(S1P)
#endif
#if !defined(MPFC_GROUP) || MPFC_GROUP == 4
MPFC_INST_TILE(S2Pin)
MPFC_INST_GEN(S2Pin)
#endif
#if !defined(MPFC_GROUP) || MPFC_GROUP == 5
MPFC_INST_TILE(F2N)
MPFC_INST_TILE(F2P)
MPFC_INST_BATCH(F2N)
MPFC_INST_BATCH(F2P)
#endif
#if !defined(MPFC_GROUP) || MPFC_GROUP == 6
MPFC_INST_TILE(F1N)
MPFC_INST_TILE(F1P)
MPFC_INST_BATCH(F1N)
MPFC_INST_BATCH(F1P)
#endif
#if !defined(MPFC_GROUP) || MPFC_GROUP == 7
MPFC_INST_TILE(Poi)
void launch_coarsest_poisson(const PoissonOp<double>& op, const CoarseArgs<double>& A,
                             const CycleState* stop, hipStream_t s) {
    hipLaunchKernelGGL((k_coarsest_poisson<double>), dim3(1), dim3(CG_THREADS), 0, s, op, A, stop);
}
#endif

}  // namespace mpfc
