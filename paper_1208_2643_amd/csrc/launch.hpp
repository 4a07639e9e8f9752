// Launchers of the fused tile kernels, the persistent coarse-level kernels and
// their batched forms (tiles.hpp).  They are declared here and defined, with
// an explicit instantiation for every operator the library uses, in
// launch_inst.hip, which the build compiles once per operator group in
// parallel; the host code calls them without instantiating the kernels itself.
#pragma once
#include <hip/hip_runtime.h>

#include "tiles.hpp"

namespace mpfc {

// Tile shapes (interior TX x TY, largest halo HMAX) instantiated for the
// tiled levels.  Shapes 0-3 serve halos up to 6 (nu <= 2), shapes 4-6 up to
// 10.  Grids with a side that is not a power of two take shapes 0 and 2.
struct TileShape { int tx, ty, hmax; };
constexpr TileShape kShapes[] = {{64, 32, 6},  {32, 32, 6},  {32, 16, 6}, {16, 16, 6},
                                 {64, 16, 10}, {32, 16, 10}, {16, 16, 10}};
constexpr int kNumShapes = 7;
constexpr bool gen_shape(int k) { return k == 0 || k == 2; }

// One tiled level: grid (m / tx, n / ty) workgroups of tile shape `shape`;
// the periodic, Neumann or general-index instantiation by A.g.
template <class Op, bool UP>
void launch_tile(const Op& op, const TileArgs<typename Op::real>& A, int shape,
                 const CycleState* stop, hipStream_t s);

// Every level from the first untiled one down, one workgroup; `four`: the
// coarsest grid has 4 cells (2 x 2), else 8 (2 x 4 or 4 x 2).
template <class Op>
void launch_coarse(const Op& op, const CoarseArgs<typename Op::real>& A, bool four,
                   const CycleState* stop, hipStream_t s);

// Coarsest level of a general grid: red-black sweeps (MPFC system) ...
template <class Op>
void launch_coarsest_gen(const Op& op, const CoarseArgs<typename Op::real>& A,
                         const CycleState* stop, hipStream_t s);
// ... and the exact separable solve of its Poisson problem.
void launch_coarsest_poisson(const PoissonOp<double>& op, const CoarseArgs<double>& A,
                             const CycleState* stop, hipStream_t s);

// Batched: one tiled level size of many grids (work list `items`), and the
// persistent coarse levels with one workgroup per grid (coarsest NC cells).
template <class Op, bool UP>
void launch_tile_batched(bool neu, int shape, const BatchTile<Op>* args, const BatchItem* items,
                         int n, hipStream_t s);
template <class Op, int NC>
void launch_coarse_batched(bool neu, int nsim, const BatchCoarse<Op>* args, hipStream_t s);

}  // namespace mpfc
