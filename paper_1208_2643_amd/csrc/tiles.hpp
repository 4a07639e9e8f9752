// Fused, LDS-tiled FAS V-cycle kernels for gfx950.
//
// Each multigrid level above 32x32 cells costs two launches per V-cycle:
//   down: complete the FAS right-hand side, nu1 red-black nonlinear
//         Gauss-Seidel passes (App. B smoother), write u, then the residual
//         and its 2x2-average restriction together with the restriction of u
//         onto the next level (one read of the level, one write);
//   up:   load u with the bilinear coarse-grid correction applied, nu2
//         passes, write u; on the finest level also the residual norm of the
//         stopping test.
// All levels of at most 32x32 cells run in one persistent single-workgroup
// kernel that keeps them in LDS and solves the coarsest grid directly.
//
// Tiles.  A workgroup owns a tx x ty interior tile and loads it with a halo
// of H cells (periodic wrap, or reflection on a Neumann axis) into LDS.  After p half-sweeps the cells at
// distance >= p from the loaded border hold exactly the values of a global
// red-black sweep (a red cell only reads black neighbours and vice versa), so
// H >= number of half-sweeps (+1 when a residual follows) makes the interior
// exact.  Output goes to a second buffer (ping-pong), so neighbouring tiles
// always read the values from before the launch.  H is even, so the loaded
// region starts on an even global index: 2x2 blocks of the loaded region are
// exactly the fine cells under one coarse cell.
//
// Threads own 2x2 blocks of the loaded region: both red cells of a block in
// red passes, both black cells in black passes, all four for the residual,
// restriction and prolongation.  Right-hand side and phi^k of owned cells
// live in registers.  LDS holds the unknowns split by colour: U[f][c][y][x/2]
// with c = (x + y) & 1, so a thread's own cells and all neighbours of one
// colour are contiguous across lanes (no bank conflicts on 8-byte accesses).
#pragma once
#include <type_traits>

#include "kernels.hpp"

namespace mpfc {

// ---------------------------------------------------------------------------
// Cell operators.  ns[f] is the sum of the four neighbours of field f.

// MPFC system N(u) = f (App. B.1 / B.2), optionally in correction (DEFECT) form.
// PIN: the pinning of Sec. 4.6 adds the per-cell weight w to the coefficient
// of phi in N^(2) (the unknown mu is mu~); w = 0 otherwise.
template <typename T, int SCHEME, bool NEWTON, bool DEFECT, bool PIN = false>
struct MpfcOp {
    using real = T;
    static constexpr int NF = 3;
    static constexpr bool XK = SCHEME == 2;
    static constexpr bool PB = DEFECT;
    static constexpr bool PW = PIN;
    LevelOp<T> op;

    __device__ __forceinline__ void apply(const T* u, const T* ns, T xk, T pb, T w, T* N) const {
        const T lphi = (ns[0] - T(4) * u[0]) * op.ih2;
        const T lmu = (ns[1] - T(4) * u[1]) * op.ih2;
        const T lka = (ns[2] - T(4) * u[2]) * op.ih2;
        const T al = PIN ? op.al + w : op.al;
        N[0] = u[0] - op.c * lmu;
        N[1] = u[1] - nl_value<T, SCHEME, DEFECT>(u[0], pb, xk) - al * u[0] - lka;
        N[2] = u[2] - op.e * lphi;
    }
    // Collective update of one cell: J_loc delta = f - N(u) (see relax_at).
    __device__ __forceinline__ void relax(T* u, const T* ns, const T* f, T xk, T pb, T w) const {
        T N[3];
        apply(u, ns, xk, pb, w, N);
        const T r1 = f[0] - N[0], r2 = f[1] - N[1], r3 = f[2] - N[2];
        // (the base phi pb exists only in correction form)
        const T d = (PIN ? op.al + w : op.al) +
                    nl_lin<T, SCHEME, NEWTON>(DEFECT ? pb + u[0] : u[0], xk);
        const T a = T(4) * op.c * op.ih2, b = T(4) * op.ih2, ec = T(4) * op.e * op.ih2;
        const T det = T(1) + a * d + a * b * ec;
        const T dm = (r2 + (d + b * ec) * r1 - b * r3) * recip_ge1(det);
        const T dx = r1 - a * dm;
        const T dk = r3 - ec * dx;
        u[0] += op.w * dx;
        u[1] += op.w * dm;
        u[2] += op.w * dk;
    }
};

// Poisson problem -Lap_h w = b (App. A "-1" norm), same interface.
template <typename T>
struct PoissonOp {
    using real = T;
    static constexpr int NF = 1;
    static constexpr bool XK = false;
    static constexpr bool PB = false;
    static constexpr bool PW = false;
    T ih2, h2;
    __device__ __forceinline__ void apply(const T* u, const T* ns, T, T, T, T* N) const {
        N[0] = (T(4) * u[0] - ns[0]) * ih2;
    }
    __device__ __forceinline__ void relax(T* u, const T* ns, const T* f, T, T, T) const {
        u[0] = T(0.25) * (h2 * f[0] + ns[0]);
    }
};

// ---------------------------------------------------------------------------
template <typename T>
struct TileArgs {
    Grid g;                 // this level
    const T* uin[3];        // u before the launch
    T* uout[3];             // u after the launch (interior cells)
    const T* f[3];          // right-hand side: complete (finest down, every up) or the
                            // restricted residual R r (coarse down, completed in-kernel)
    T* fout[3];             // coarse down: completed right-hand side f = R r + N(u)
    const T* xk;            // phi^k on this level (scheme 2)
    const T* pb;            // base phi (correction form)
    T* uH[3]; T* vH[3]; T* rH[3];          // down: restricted u (twice) and residual
    T* xkH; T* pbH;         // down (nullable): 2x2 averages of phi^k and of the base phi
    const T* pin;           // pinning weight on this level (Op::PW)
    const T* cuH[3]; const T* cvH[3];      // up: coarse u after and before its solve
    int complete_f;         // down on a coarse level
    int zero_in;            // u before the launch is zero (uin is not read)
    int nsweep;             // red-black half-sweeps (2 nu)
    int H;                  // halo (even)
    int tx, ty;             // interior tile (even, divides m, n)
    // residual norm (finest up): per-block FP64 sums of r^2 into part[]
    int norm;
    double* part;
};

template <typename T>
__device__ __forceinline__ T bilinear(const T* __restrict__ uH, const T* __restrict__ vH, int I,
                                      int J, int Is, int Js, int mc) {
    const size_t a = (size_t)J * mc + I, b = (size_t)J * mc + Is;
    const size_t c = (size_t)Js * mc + I, d = (size_t)Js * mc + Is;
    return T(9.0 / 16.0) * (uH[a] - vH[a]) +
           T(3.0 / 16.0) * ((uH[b] - vH[b]) + (uH[c] - vH[c])) +
           T(1.0 / 16.0) * (uH[d] - vH[d]);
}

// Cell index along one axis inside the tile and coarse kernels: plain
// wrap-around in the periodic instantiation (NEU = false), the per-axis ghost
// rule (axis_index) in the instantiation for grids with a Neumann axis.
// GEN: instantiation for grids whose sides need not be powers of two.
template <bool NEU, bool GEN = false>
__device__ __forceinline__ int bidx(int i, int m, int neumann_axis) {
    if constexpr (GEN) return axis_index_any(i, m, NEU && neumann_axis);
    else if constexpr (NEU) return axis_index(i, m, neumann_axis);
    else return i & (m - 1);
}
template <bool GEN>
__device__ __forceinline__ size_t tat(int i, int j, const Grid& g) {
    if constexpr (GEN) return (size_t)j * (size_t)g.m + (size_t)i;
    else return ((size_t)j << g.lm) + (size_t)i;
}

// XCD-aware order of nt work items: workgroups are dealt round-robin to the 8
// XCDs, each with its own L2.  Workgroup b (on XCD b % 8) takes item
// (b % 8) * (nt / 8) + b / 8, so every XCD sweeps one contiguous strip of
// tiles and the halos it re-reads are mostly in its own L2.
__device__ __forceinline__ int xcd_item(int b, int nt) {
    return (nt & 7) == 0 ? (b & 7) * (nt >> 3) + (b >> 3) : b;
}

#ifndef MPFC_TILE_THREADS
#define MPFC_TILE_THREADS 512
#endif
// Threads of a tile workgroup.
constexpr int kTileThreads = MPFC_TILE_THREADS;

// One tile of a tiled level, in phases:
//   load_direct  u (tile + halo) and, for up launches, u_H - v_H over the
//                tile's coarse footprint, from global memory into LDS;
//   fetch_rhs    the right-hand side and coefficients of the owned blocks
//                into registers;
//   compute      prolongation (up), completion of the coarse right-hand side
//                (coarse down), the red-black passes, the store of u, and the
//                residual with its restriction (down) or norm (finest up).
// EXACT: the launch's tile is the shape's (A.tx = TX, A.ty = TY) and its halo
// the shape's allowance (A.H = HMAX), so every extent is a compile-time
// constant.
template <class Op, int TX, int TY, int HMAX, bool UP, bool NEU, bool GEN, bool EXACT>
struct TileWork {
    using T = typename Op::real;
    static constexpr int NF = Op::NF;
    static constexpr int NT = kTileThreads;
    static constexpr int LX2M = (TX + 2 * HMAX) / 2;
    static constexpr int LYM = TY + 2 * HMAX;
    static constexpr int SL = (LX2M * (LYM / 2) + NT - 1) / NT;  // owned blocks per thread
    // LDS row length (doubles per colour and row), padded so that a wave's
    // consecutive blocks continue across a block-row break on the next banks:
    // the block-row stride 2 P equals LX2 modulo the 32 doubles of a bank cycle.
    static constexpr int pad_row(int l) {
        int p = l;
        while (((2 * p - l) % 32 + 32) % 32 != 0) ++p;
        return p;
    }
    static constexpr int LXP = pad_row(LX2M);
    static constexpr int CXM = LX2M + 2, CYM = LYM / 2 + 2;       // coarse footprint

    struct Lds {
        T U[NF][2][LYM][LXP];
        T E[UP ? NF : 1][UP ? CYM : 1][UP ? CXM : 1];  // up: uH - vH
        double red[NT / 64];
    };
    // Extents of the tile (tbx, tby) of a launch.
    struct Geo {
        int H, tx, ty, LX, LY, LX2, nblk, x0, y0, tbx, tby;
    };
    // Right-hand side and coefficients of the owned blocks' four cells (cell
    // order: (0,0) (1,1) red, (1,0) (0,1) black).
    struct Rhs {
        T f[SL][4][NF];
        T xk[SL][4];
        T pb[SL][4];
        T w[SL][4];
    };
    // OWN (a thread owns at most one block): the block's four cells are also
    // kept in registers, updated together with LDS.  Two of each cell's four
    // neighbours lie in its own block, so half of the neighbour reads come
    // from registers and LDS traffic per relaxation halves.  Only the owner
    // writes a cell (except the Neumann ghost restore, after which the copy
    // is reloaded).
    static constexpr bool OWN = SL == 1;
    struct Own {
        T u[4][NF];
    };
    // cell offsets within a block: 0 = (0,0), 1 = (1,1) red; 2 = (1,0), 3 = (0,1) black
    static constexpr int cdx(int c) { return (c == 1 || c == 2) ? 1 : 0; }
    static constexpr int cdy(int c) { return (c == 1 || c == 3) ? 1 : 0; }
    static constexpr int cid(int dx, int dy) { return dx == dy ? dx : (dx ? 2 : 3); }

    // Neighbour sums of cell C of the owned block (bx, by), every field, in
    // the order (east + west) + (north + south): own-block neighbours from
    // registers, the others from LDS.
    // Indices are clamped to the loaded region: a cell on its border gets a
    // meaningless sum, and its result is discarded by the caller.
    template <int C>
    static __device__ __forceinline__ void nsum_own(const Lds& S, const Own& O, const Geo& G,
                                                    int bx, int by, T (&ns)[NF]) {
        constexpr int dx = cdx(C), dy = cdy(C), oc = ((dx + dy) & 1) ^ 1;
        const int y = 2 * by + dy;
        const int ke = min(bx + 1, G.LX2 - 1), kw = max(bx - 1, 0);
        const int yn = min(y + 1, G.LY - 1), ys = max(y - 1, 0);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const T e = dx == 0 ? O.u[cid(1, dy)][f] : S.U[f][oc][y][ke];
            const T w = dx == 1 ? O.u[cid(0, dy)][f] : S.U[f][oc][y][kw];
            const T n = dy == 0 ? O.u[cid(dx, 1)][f] : S.U[f][oc][yn][bx];
            const T s = dy == 1 ? O.u[cid(dx, 0)][f] : S.U[f][oc][ys][bx];
            ns[f] = (e + w) + (n + s);
        }
    }
    // The owned block's cells from LDS into registers (after a barrier).
    static __device__ __forceinline__ void load_own(const Lds& S, const Geo& G, Own& O) {
        const int b = threadIdx.x;
        if (b >= G.nblk) return;
        const int by = b / G.LX2, bx = b - by * G.LX2;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int y = 2 * by + cdy(c);
#pragma unroll
            for (int f = 0; f < NF; ++f) O.u[c][f] = S.U[f][(cdx(c) + cdy(c)) & 1][y][bx];
        }
    }

    static __device__ __forceinline__ Geo geo(const TileArgs<T>& A, int tbx, int tby) {
        Geo G;
        G.H = EXACT ? HMAX : A.H;
        G.tx = EXACT ? TX : A.tx;
        G.ty = EXACT ? TY : A.ty;
        G.LX = G.tx + 2 * G.H;
        G.LY = G.ty + 2 * G.H;
        G.LX2 = G.LX >> 1;
        G.nblk = G.LX2 * (G.LY >> 1);
        G.x0 = tbx * G.tx - G.H;
        G.y0 = tby * G.ty - G.H;
        G.tbx = tbx;
        G.tby = tby;
        return G;
    }

    static __device__ __forceinline__ size_t cell(const Grid& g, int x, int y) {
        return tat<GEN>(bidx<NEU, GEN>(x, g.m, g.bc & BC_NEUMANN_X),
                        bidx<NEU, GEN>(y, g.n, g.bc & BC_NEUMANN_Y), g);
    }
    static __device__ __forceinline__ size_t coarse_cell(const Grid& g, int cx, int cy) {
        const int mc = g.m >> 1, nc = g.n >> 1;
        return (size_t)bidx<NEU, GEN>(cy, nc, g.bc & BC_NEUMANN_Y) * mc +
               bidx<NEU, GEN>(cx, mc, g.bc & BC_NEUMANN_X);
    }

    static __device__ __forceinline__ void fetch_rhs(const TileArgs<T>& A, const Geo& G, Rhs& R) {
        const Grid g = A.g;
        const int t = threadIdx.x;
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int b = t + s * NT;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
#pragma unroll
                for (int f = 0; f < NF; ++f) R.f[s][c][f] = T(0);
                R.xk[s][c] = T(0);
                R.pb[s][c] = T(0);
                R.w[s][c] = T(0);
            }
            if (b >= G.nblk) continue;
            const int by = b / G.LX2, bx = b - by * G.LX2;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int dx = (c == 1 || c == 2) ? 1 : 0, dy = (c == 1 || c == 3) ? 1 : 0;
                const int x = 2 * bx + dx, y = 2 * by + dy;
                if (x < 1 || y < 1 || x >= G.LX - 1 || y >= G.LY - 1) continue;  // never updated
                const size_t gq = cell(g, G.x0 + x, G.y0 + y);
                if constexpr (Op::XK) R.xk[s][c] = A.xk[gq];
                if constexpr (Op::PB) R.pb[s][c] = A.pb[gq];
                if constexpr (Op::PW) R.w[s][c] = A.pin[gq];
#pragma unroll
                for (int f = 0; f < NF; ++f) R.f[s][c][f] = A.f[f][gq];
            }
        }
    }

    // u (tile + halo) and, up, uH - vH into LDS, coalesced along rows; a
    // barrier must follow.
    // Loads of LCH consecutive strides are issued together, so a thread waits
    // once per LCH strides rather than once per stride.  Indices past the end
    // are clamped to the last cell, for the load and the store alike (the
    // same value stored twice), so no load sits behind a branch.
    static constexpr int LCH = 4;
    // `mid` runs once the first stride group's loads are issued (before any of
    // them is waited for): the caller requests the right-hand side there.
    template <class Mid>
    static __device__ __forceinline__ void load_direct(const TileArgs<T>& A, const Geo& G, Lds& S,
                                                       Mid&& mid) {
        const Grid g = A.g;
        const int t = threadIdx.x;
        const int total = G.LX * G.LY;
        constexpr int NLD = (2 * LX2M * LYM + NT - 1) / NT;  // strides of the largest tile
        // up: u_H - v_H over the tile's coarse footprint, requested first so
        // that its loads are in flight together with the tile's
        constexpr int NE = UP ? (CXM * CYM + NT - 1) / NT : 1;
        T ev[NE][NF];
        int exs[NE], eys[NE];
        if constexpr (UP) {
            const int CX = G.LX2 + 2, CY = (G.LY >> 1) + 2, ctot = CX * CY;
            const int cx0 = (G.x0 >> 1) - 1, cy0 = (G.y0 >> 1) - 1;
            (void)CY;
#pragma unroll
            for (int j = 0; j < NE; ++j) {
                const int q = min(t + j * NT, ctot - 1);
                eys[j] = q / CX;
                exs[j] = q - eys[j] * CX;
                const size_t gq = coarse_cell(g, cx0 + exs[j], cy0 + eys[j]);
#pragma unroll
                for (int f = 0; f < NF; ++f) ev[j][f] = A.cuH[f][gq] - A.cvH[f][gq];
            }
        }
        if (A.zero_in) {
            mid();
            for (int q = t; q < total; q += NT) {
                const int y = q / G.LX, x = q - y * G.LX;
#pragma unroll
                for (int f = 0; f < NF; ++f) S.U[f][(x + y) & 1][y][x >> 1] = T(0);
            }
        } else {
#pragma unroll
            for (int k0 = 0; k0 < NLD; k0 += LCH) {
                T v[LCH][NF];
                int xs[LCH], ys[LCH];
#pragma unroll
                for (int j = 0; j < LCH; ++j) {
                    if (k0 + j >= NLD) break;
                    const int q = min(t + (k0 + j) * NT, total - 1);
                    ys[j] = q / G.LX;
                    xs[j] = q - ys[j] * G.LX;
                    const size_t gq = cell(g, G.x0 + xs[j], G.y0 + ys[j]);
#pragma unroll
                    for (int f = 0; f < NF; ++f) v[j][f] = A.uin[f][gq];
                }
                if (k0 == 0) mid();
#pragma unroll
                for (int j = 0; j < LCH; ++j) {
                    if (k0 + j >= NLD) break;
                    const int x = xs[j], y = ys[j];
#pragma unroll
                    for (int f = 0; f < NF; ++f) S.U[f][(x + y) & 1][y][x >> 1] = v[j][f];
                }
            }
        }
        if constexpr (UP) {
#pragma unroll
            for (int j = 0; j < NE; ++j)
#pragma unroll
                for (int f = 0; f < NF; ++f) S.E[f][eys[j]][exs[j]] = ev[j][f];
        }
    }

    // Everything after the tile is in LDS (entered after a barrier).  `pslot`
    // is where the workgroup's residual sum goes in A.part.
    static __device__ __forceinline__ void compute(const Op& op, const TileArgs<T>& A,
                                                   const Geo& G, Lds& S, Rhs& R, int pslot) {
        const Grid g = A.g;
        const int H = G.H, tx = G.tx, ty = G.ty, LX = G.LX, LY = G.LY, LX2 = G.LX2;
        const int nblk = G.nblk, x0 = G.x0, y0 = G.y0, tbx = G.tbx, tby = G.tby;
        const int t = threadIdx.x;
        auto& U = S.U;
        auto& E = S.E;
        auto& red = S.red;
        auto& fr = R.f;
        const auto& xkr = R.xk;
        const auto& pbr = R.pb;
        const auto& wr = R.w;
        Own O;
        if constexpr (OWN && !UP) load_own(S, G, O);
    // 3. up: add the coarse-grid correction P(uH - vH) to every loaded cell
    //    (uH - vH over the tile's coarse footprint, one coarse cell of margin,
    //    staged in LDS).
    if constexpr (UP && OWN) {
        // the block's 3x3 coarse neighbourhood once per field, then its four cells
        if (t < nblk) {
            const int by = t / LX2, bx = t - by * LX2;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                T e9[3][3];
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int i = 0; i < 3; ++i) e9[j][i] = E[f][by + j][bx + i];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int dx = cdx(c), dy = cdy(c);
                    const int x = 2 * bx + dx, y = 2 * by + dy;
                    const int si = dx ? 2 : 0, sj = dy ? 2 : 0;
                    const T v = U[f][(x + y) & 1][y][x >> 1] +
                                (T(9.0 / 16.0) * e9[1][1] +
                                 T(3.0 / 16.0) * (e9[1][si] + e9[sj][1]) +
                                 T(1.0 / 16.0) * e9[sj][si]);
                    U[f][(x + y) & 1][y][x >> 1] = v;
                    O.u[c][f] = v;
                }
            }
        }
        __syncthreads();
    } else if constexpr (UP) {
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int b = t + s * NT;
            if (b >= nblk) continue;
            const int by = b / LX2, bx = b - by * LX2;
            const int cx = bx + 1, cy = by + 1;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int dx = (c == 1 || c == 2) ? 1 : 0, dy = (c == 1 || c == 3) ? 1 : 0;
                const int x = 2 * bx + dx, y = 2 * by + dy;
                const int sx = dx ? cx + 1 : cx - 1, sy = dy ? cy + 1 : cy - 1;
#pragma unroll
                for (int f = 0; f < NF; ++f)
                    U[f][(x + y) & 1][y][x >> 1] +=
                        T(9.0 / 16.0) * E[f][cy][cx] +
                        T(3.0 / 16.0) * (E[f][cy][sx] + E[f][sy][cx]) +
                        T(1.0 / 16.0) * E[f][sy][sx];
            }
        }
        __syncthreads();
    }

    // 3'. coarse down: f = R r + N(u) at every cell that can be updated.
    if (!UP && OWN && A.complete_f) {
        if (t < nblk) {
            const int by = t / LX2, bx = t - by * LX2;
            // all four cells computed without branches (the chains
            // interleave), kept only where the cell can be updated
            auto cell_f = [&](auto cc_) {
                constexpr int c = decltype(cc_)::value;
                const int x = 2 * bx + cdx(c), y = 2 * by + cdy(c);
                const bool in = x >= 1 && y >= 1 && x < LX - 1 && y < LY - 1;
                T ns[NF], N[NF];
                nsum_own<c>(S, O, G, bx, by, ns);
                op.apply(O.u[c], ns, xkr[0][c], pbr[0][c], wr[0][c], N);
#pragma unroll
                for (int f = 0; f < NF; ++f) fr[0][c][f] = in ? fr[0][c][f] + N[f] : fr[0][c][f];
            };
            cell_f(std::integral_constant<int, 0>{});
            cell_f(std::integral_constant<int, 1>{});
            cell_f(std::integral_constant<int, 2>{});
            cell_f(std::integral_constant<int, 3>{});
        }
        __syncthreads();
    } else if (!UP && A.complete_f) {
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int b = t + s * NT;
            if (b >= nblk) continue;
            const int by = b / LX2, bx = b - by * LX2;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int dx = (c == 1 || c == 2) ? 1 : 0, dy = (c == 1 || c == 3) ? 1 : 0;
                const int x = 2 * bx + dx, y = 2 * by + dy;
                if (x < 1 || y < 1 || x >= LX - 1 || y >= LY - 1) continue;
                const int col = (x + y) & 1, oc = col ^ 1, k = x >> 1;
                const int ke = (x + 1) >> 1, kw = (x - 1) >> 1;
                T u[NF], ns[NF], N[NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    u[f] = U[f][col][y][k];
                    ns[f] = (U[f][oc][y][ke] + U[f][oc][y][kw]) +
                            (U[f][oc][y + 1][k] + U[f][oc][y - 1][k]);
                }
                op.apply(u, ns, xkr[s][c], pbr[s][c], wr[s][c], N);
#pragma unroll
                for (int f = 0; f < NF; ++f) fr[s][c][f] += N[f];
            }
        }
        // every N(u) above reads u as loaded: no pass may write before all
        // waves are done (waves with a second owned block finish later)
        __syncthreads();
    }

    // 4. red-black passes; pass p is exact on cells at distance >= p.  The
    //    colour is a compile-time constant inside `pass`, so the per-cell
    //    register arrays are indexed statically.
    auto pass = [&](auto colc, int p) {
        constexpr int colour = decltype(colc)::value;
        constexpr int oc = colour ^ 1;
        if constexpr (OWN) {
            if (t >= nblk) return;
            const int by = t / LX2, bx = t - by * LX2;
            // both cells of the colour are relaxed without branches (their
            // chains interleave; they do not neighbour each other), then
            // stored where the pass updates them
            auto cell = [&](auto cc_, T (&u)[NF]) {
                constexpr int c = decltype(cc_)::value;
                T ns[NF];
                nsum_own<c>(S, O, G, bx, by, ns);
#pragma unroll
                for (int f = 0; f < NF; ++f) u[f] = O.u[c][f];
                op.relax(u, ns, fr[0][c], xkr[0][c], pbr[0][c], wr[0][c]);
            };
            // (a cell the pass does not update gets its own value back: only
            // its owner writes it, so the store is branch-free)
            auto put = [&](auto cc_, const T (&u)[NF]) {
                constexpr int c = decltype(cc_)::value;
                const int x = 2 * bx + cdx(c), y = 2 * by + cdy(c);
                const bool in = x >= p && y >= p && x < LX - p && y < LY - p;
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const T v = in ? u[f] : O.u[c][f];
                    U[f][colour][y][bx] = v;
                    O.u[c][f] = v;
                }
            };
            constexpr int c0 = colour == 0 ? 0 : 2, c1 = colour == 0 ? 1 : 3;
            T u0[NF], u1[NF];
            cell(std::integral_constant<int, c0>{}, u0);
            cell(std::integral_constant<int, c1>{}, u1);
            put(std::integral_constant<int, c0>{}, u0);
            put(std::integral_constant<int, c1>{}, u1);
            return;
        }
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int b = t + s * NT;
            if (b >= nblk) continue;
            const int by = b / LX2, bx = b - by * LX2;
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
                const int c = colour == 0 ? cc : 2 + cc;
                const int dx = (c == 1 || c == 2) ? 1 : 0, dy = (c == 1 || c == 3) ? 1 : 0;
                const int x = 2 * bx + dx, y = 2 * by + dy;
                if (x < p || y < p || x >= LX - p || y >= LY - p) continue;
                const int k = x >> 1, ke = (x + 1) >> 1, kw = (x - 1) >> 1;
                T u[NF], ns[NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    u[f] = U[f][colour][y][k];
                    ns[f] = (U[f][oc][y][ke] + U[f][oc][y][kw]) +
                            (U[f][oc][y + 1][k] + U[f][oc][y - 1][k]);
                }
                op.relax(u, ns, fr[s][c], xkr[s][c], pbr[s][c], wr[s][c]);
#pragma unroll
                for (int f = 0; f < NF; ++f) U[f][colour][y][k] = u[f];
            }
        }
    };
    // Neumann boundaries: halo cells outside the grid hold the even reflection
    // of interior cells (App. A ghost rule, extended through the halo).  A pass
    // also relaxes them as if they were cells; afterwards they are restored
    // from their mirror cells, x first, then y (corners get both reflections),
    // so every relaxed grid cell reads ghosts equal to its mirror's value from
    // before the pass, as in a global sweep.
    const bool mir_x = NEU && (g.bc & BC_NEUMANN_X) && (x0 < 0 || x0 + LX > g.m);
    const bool mir_y = NEU && (g.bc & BC_NEUMANN_Y) && (y0 < 0 || y0 + LY > g.n);
    auto restore_ghosts = [&]() {
        if (mir_x) {
            for (int q = t; q < 2 * H * LY; q += NT) {
                const int y = q / (2 * H), k = q - y * (2 * H);
                const int x = k < H ? k : LX - 2 * H + k;
                const int gx = x0 + x;
                if (gx >= 0 && gx < g.m) continue;
                const int xm = (GEN ? axis_index_any(gx, g.m, true) : axis_index(gx, g.m, true)) - x0;
#pragma unroll
                for (int f = 0; f < NF; ++f)
                    U[f][(x + y) & 1][y][x >> 1] = U[f][(xm + y) & 1][y][xm >> 1];
            }
            __syncthreads();
        }
        if (mir_y) {
            for (int q = t; q < 2 * H * LX; q += NT) {
                const int k = q / LX, x = q - k * LX;
                const int y = k < H ? k : LY - 2 * H + k;
                const int gy = y0 + y;
                if (gy >= 0 && gy < g.n) continue;
                const int ym = (GEN ? axis_index_any(gy, g.n, true) : axis_index(gy, g.n, true)) - y0;
#pragma unroll
                for (int f = 0; f < NF; ++f)
                    U[f][(x + y) & 1][y][x >> 1] = U[f][(x + ym) & 1][ym][x >> 1];
            }
            __syncthreads();
        }
    };
    for (int p = 1; p <= A.nsweep; ++p) {
        if (((p - 1) & 1) == 0) pass(std::integral_constant<int, 0>{}, p);
        else pass(std::integral_constant<int, 1>{}, p);
        __syncthreads();
        if constexpr (NEU) {
            restore_ghosts();
            if constexpr (OWN)
                if (mir_x || mir_y) load_own(S, G, O);
        }
    }

    // 5. interior u back to global memory, coalesced along rows.
    const int gx0 = tbx * tx, gy0 = tby * ty;
    for (int q = t; q < tx * ty; q += NT) {
        const int yi = q / tx, xi = q - yi * tx;
        const int x = xi + H, y = yi + H;
        const size_t gq = tat<GEN>(gx0 + xi, gy0 + yi, g);
#pragma unroll
        for (int f = 0; f < NF; ++f) A.uout[f][gq] = U[f][(x + y) & 1][y][x >> 1];
    }

    // 6. interior blocks: residual; down restricts it (and u), finest up sums r^2.
    double acc = 0.0;
    const int mc = g.m >> 1;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int b = t + s * NT;
        if (b >= nblk) continue;
        const int by = b / LX2, bx = b - by * LX2;
        if (2 * bx < H || 2 * bx >= H + tx || 2 * by < H || 2 * by >= H + ty) continue;
        if (UP && !A.norm) continue;
        T su[NF], sr[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) { su[f] = T(0); sr[f] = T(0); }
        auto res_own = [&](auto cc_) {
            constexpr int c = decltype(cc_)::value;
            T ns[NF], N[NF];
            nsum_own<c>(S, O, G, bx, by, ns);
            op.apply(O.u[c], ns, xkr[0][c], pbr[0][c], wr[0][c], N);
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const T r = fr[0][c][f] - N[f];
                su[f] += O.u[c][f];
                sr[f] += r;
                acc += (double)r * (double)r;
            }
        };
        if constexpr (OWN) {
            res_own(std::integral_constant<int, 0>{});
            res_own(std::integral_constant<int, 1>{});
            res_own(std::integral_constant<int, 2>{});
            res_own(std::integral_constant<int, 3>{});
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int dx = (c == 1 || c == 2) ? 1 : 0, dy = (c == 1 || c == 3) ? 1 : 0;
                const int x = 2 * bx + dx, y = 2 * by + dy;
                const int col = (x + y) & 1, oc = col ^ 1, k = x >> 1;
                const int ke = (x + 1) >> 1, kw = (x - 1) >> 1;
                T u[NF], ns[NF], N[NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    u[f] = U[f][col][y][k];
                    ns[f] = (U[f][oc][y][ke] + U[f][oc][y][kw]) +
                            (U[f][oc][y + 1][k] + U[f][oc][y - 1][k]);
                }
                op.apply(u, ns, xkr[s][c], pbr[s][c], wr[s][c], N);
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const T r = fr[s][c][f] - N[f];
                    su[f] += u[f];
                    sr[f] += r;
                    acc += (double)r * (double)r;
                }
            }
        }
        if constexpr (!UP) {
            const int I = (gx0 + 2 * bx - H) >> 1, J = (gy0 + 2 * by - H) >> 1;
            const size_t Q = (size_t)J * mc + I;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const T avg = T(0.25) * su[f];
                A.uH[f][Q] = avg;
                A.vH[f][Q] = avg;
                A.rH[f][Q] = T(0.25) * sr[f];
            }
            // coefficient fields of the coarse level, in the order of additions
            // of a plain 2x2 average: ((f00 + f10) + (f01 + f11)) / 4
            if constexpr (Op::XK)
                if (A.xkH) A.xkH[Q] = T(0.25) * ((xkr[s][0] + xkr[s][2]) + (xkr[s][3] + xkr[s][1]));
            if constexpr (Op::PB)
                if (A.pbH) A.pbH[Q] = T(0.25) * ((pbr[s][0] + pbr[s][2]) + (pbr[s][3] + pbr[s][1]));
        }
    }
    if constexpr (!UP) {
        // completed coarse-level right-hand side for the up launch
        if (A.complete_f) {
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const int b = t + s * NT;
                if (b >= nblk) continue;
                const int by = b / LX2, bx = b - by * LX2;
                if (2 * bx < H || 2 * bx >= H + tx || 2 * by < H || 2 * by >= H + ty) continue;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int dx = (c == 1 || c == 2) ? 1 : 0, dy = (c == 1 || c == 3) ? 1 : 0;
                    const size_t gq = tat<GEN>(gx0 + 2 * bx - H + dx, gy0 + 2 * by - H + dy, g);
#pragma unroll
                    for (int f = 0; f < NF; ++f) A.fout[f][gq] = fr[s][c][f];
                }
            }
        }
    } else {
        if (A.norm) {
            // per-block sum of r^2; k_norm_finalize adds them and decides
            const double bs = block_sum<NT>(acc, red);
            if (t == 0) A.part[pslot] = bs;
        }
    }
    }
};

// Body of one tile launch: the tile into LDS, its right-hand side into
// registers, then the computation.
template <class Op, int TX, int TY, int HMAX, bool UP, bool NEU, bool GEN = false,
          bool EXACT = false>
__device__ __forceinline__ void tile_body(const Op& op, const TileArgs<typename Op::real>& A,
                                          const CycleState* stop, int tbx, int tby, int pslot) {
    using W = TileWork<Op, TX, TY, HMAX, UP, NEU, GEN, EXACT>;
    __shared__ typename W::Lds S;
    if (stopped(stop)) return;
    const typename W::Geo G = W::geo(A, tbx, tby);
    typename W::Rhs R;
    if constexpr (UP) {
        // the right-hand side is first used after the prolongation, which
        // covers its latency
        W::load_direct(A, G, S, [] {});
        __syncthreads();
        W::fetch_rhs(A, G, R);
    } else {
        W::load_direct(A, G, S, [&] { W::fetch_rhs(A, G, R); });
        __syncthreads();
    }
    W::compute(op, A, G, S, R, pslot);
}

// One level of one grid.  Grid: (m / tx, n / ty) workgroups of kTileThreads
// threads (tx, ty divide m, n).
template <class Op, int TX, int TY, int HMAX, bool UP, bool NEU, bool GEN = false,
          bool EXACT = false>
__global__ void __launch_bounds__(kTileThreads) k_tile(Op op, TileArgs<typename Op::real> A,
                                                       const CycleState* stop) {
    const int nt = gridDim.x * gridDim.y;
    const int tl = xcd_item(blockIdx.y * gridDim.x + blockIdx.x, nt);
    const int tby = tl / gridDim.x, tbx = tl - tby * gridDim.x;
    tile_body<Op, TX, TY, HMAX, UP, NEU, GEN, EXACT>(op, A, stop, tbx, tby, tl);
}

// Batched launch: one level of many independent grids.  Each (grid, level)
// has its own arguments, operator constants and stop flag; the work list
// holds one entry per tile.
template <class Op>
struct BatchTile {
    Op op;
    TileArgs<typename Op::real> A;
    const CycleState* stop;
    int part_off;         // first slot of this grid's residual sums in A.part
    int ntx;              // tiles in x
};

struct BatchItem {
    int arg;              // index into the BatchTile array
    int tile;             // linear tile index within that grid level
};

template <class Op, int TX, int TY, int HMAX, bool UP, bool NEU>
__global__ void __launch_bounds__(kTileThreads) k_tile_batched(const BatchTile<Op>* __restrict__ args,
                                                      const BatchItem* __restrict__ items,
                                                      int nitems) {
    const int b = xcd_item(blockIdx.x, nitems);
    const BatchItem it = items[b];
    const BatchTile<Op>& BA = args[it.arg];
    const int tby = it.tile / BA.ntx, tbx = it.tile - tby * BA.ntx;
    tile_body<Op, TX, TY, HMAX, UP, NEU>(BA.op, BA.A, BA.stop, tbx, tby, BA.part_off + it.tile);
}

// ---------------------------------------------------------------------------
// Persistent kernel: every level of at most CP_CELLS cells, in LDS, one
// workgroup.  Same V(nu1, nu2) cycle as the tiled levels; the coarsest grid is
// solved directly (CoarseSolve).
constexpr int CP_CELLS = 1024;  // largest level handled here (32 x 32)
constexpr int CP_TOTAL = 1368;  // cells of all its levels (1024 + 256 + 64 + 16 + 4, padded)
constexpr int CP_MAXLEV = 12;
constexpr int CP_THREADS = 512;  // threads of the persistent workgroup

struct CoarseGeom {
    int bc;               // boundary conditions (BC_NEUMANN_X | BC_NEUMANN_Y bits)
    int nlev;             // levels in this kernel (top first)
    int m[CP_MAXLEV], n[CP_MAXLEV], lm[CP_MAXLEV];
    int off[CP_MAXLEV];   // cell offset of each level in the LDS arrays
};

template <typename T>
struct CoarseArgs {
    CoarseGeom geo;
    T* u[3];              // top level u (in/out, global)
    const T* rr[3];       // top level restricted residual R r (global)
    const T* xk;          // phi^k on the top level (global)
    const T* pb;          // base phi on the top level (global)
    const T* pin;         // pinning weight on the top level (global; Op::PW)
    T h_top;              // spacing of the top level
    int nsw1, nsw2;       // half-sweeps down / up
    int complete_top;     // 1: rr holds R r (add N(u)); 0: rr is already the full f
    const double* G;      // Poisson: Green's matrix of the coarsest grid
    int newton_maxit;
    T newton_tol;
};

// Coarsest grid, MPFC: eliminate kappa and mu (kappa = f3 + e Lap phi,
// mu = f2 + g(phi) + al phi + Lap kappa) and solve the remaining equation
//   phi - c Lap(g(phi) + al phi + e Lap^2 phi) = f1 + c Lap(f2 + Lap f3)
// by Newton with Gaussian elimination (NC <= 8 unknowns), one thread.  Its
// solution is the unique solution of the three-field system.  Every array is
// indexed with compile-time indices only (row swaps are selects), so that it
// lives in registers.
template <class Op, int NC>
__device__ __forceinline__ void coarse_solve_mpfc(const Op& op, typename Op::real* phi,
                                                  typename Op::real* mu, typename Op::real* ka,
                                                  const typename Op::real (&f)[3 * NC],
                                                  const typename Op::real* xk,
                                                  const typename Op::real* pb,
                                                  const typename Op::real* pw, int m, int lm,
                                                  int n, int bc, int maxit, typename Op::real tol) {
    using T = typename Op::real;
    const T c = op.op.c, e = op.op.e, al = op.op.al;
    // Laplacian matrix of the m x n grid with its ghost rule (periodic: a
    // 2-cell direction couples each cell twice to its one neighbour; Neumann:
    // the ghost beside a boundary cell is that cell itself).
    const bool nx = bc & BC_NEUMANN_X, ny = bc & BC_NEUMANN_Y;
    T L[NC][NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) {
        const int i = a & (m - 1), j = a >> lm;
        const int e0 = axis_index(i + 1, m, nx) + (j << lm);
        const int e1 = axis_index(i - 1, m, nx) + (j << lm);
        const int e2 = i + (axis_index(j + 1, n, ny) << lm);
        const int e3 = i + (axis_index(j - 1, n, ny) << lm);
#pragma unroll
        for (int b = 0; b < NC; ++b) {
            const int k = (b == a ? -4 : 0) + (b == e0) + (b == e1) + (b == e2) + (b == e3);
            L[a][b] = T(k) * op.op.ih2;
        }
    }
    auto lap = [&](const T (&v)[NC], T (&out)[NC]) {
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            T s = 0;
#pragma unroll
            for (int b = 0; b < NC; ++b) s += L[a][b] * v[b];
            out[a] = s;
        }
    };
    T f1[NC], f2[NC], f3[NC], t1[NC], t2[NC], rhs[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) { f1[a] = f[a]; f2[a] = f[NC + a]; f3[a] = f[2 * NC + a]; }
    // rhs = f1 + c Lap(f2 + Lap f3)
    lap(f3, t1);
#pragma unroll
    for (int a = 0; a < NC; ++a) t1[a] += f2[a];
    lap(t1, t2);
#pragma unroll
    for (int a = 0; a < NC; ++a) rhs[a] = f1[a] + c * t2[a];
    // L3 = Lap^3 (constant part of the Jacobian)
    T L3[NC][NC];
#pragma unroll
    for (int b = 0; b < NC; ++b) {
        T col[NC], l1[NC];
#pragma unroll
        for (int a = 0; a < NC; ++a) col[a] = L[a][b];
        lap(col, l1);
        lap(l1, col);
#pragma unroll
        for (int a = 0; a < NC; ++a) L3[a][b] = col[a];
    }
    T x[NC], xkv[NC], pbv[NC], alv[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) {
        x[a] = phi[a];
        xkv[a] = Op::XK ? xk[a] : T(0);
        pbv[a] = Op::PB ? pb[a] : T(0);
        alv[a] = Op::PW ? al + pw[a] : al;  // pinning: W added to the phi coefficient
    }
    for (int it = 0; it < maxit; ++it) {
        // residual R = x - c Lap(g(x) + al x + e Lap^2 x) - rhs
        T w[NC], d[NC], R[NC], J[NC][NC + 1];
        lap(x, t1);
        lap(t1, t2);
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            w[a] = nl_value<T, (Op::XK ? 2 : 1), Op::PB>(x[a], pbv[a], xkv[a]) + alv[a] * x[a] + e * t2[a];
            d[a] = nl_lin<T, (Op::XK ? 2 : 1), true>(pbv[a] + x[a], xkv[a]) + alv[a];
        }
        lap(w, t1);
#pragma unroll
        for (int a = 0; a < NC; ++a) R[a] = x[a] - c * t1[a] - rhs[a];
        // Jacobian J = I - c (Lap diag(d) + e Lap^3), augmented with -R
#pragma unroll
        for (int a = 0; a < NC; ++a) {
#pragma unroll
            for (int b = 0; b < NC; ++b)
                J[a][b] = (a == b ? T(1) : T(0)) - c * (L[a][b] * d[b] + e * L3[a][b]);
            J[a][NC] = -R[a];
        }
        // Gaussian elimination with partial pivoting (one division per pivot)
        T ip[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
#pragma unroll
            for (int r = k + 1; r < NC; ++r) {
                const bool sw = fabs(J[r][k]) > fabs(J[k][k]);
#pragma unroll
                for (int cc = k; cc <= NC; ++cc) {
                    const T hi = J[k][cc], lo = J[r][cc];
                    J[k][cc] = sw ? lo : hi;
                    J[r][cc] = sw ? hi : lo;
                }
            }
            ip[k] = T(1) / J[k][k];
#pragma unroll
            for (int r = k + 1; r < NC; ++r) {
                const T fct = J[r][k] * ip[k];
#pragma unroll
                for (int cc = k; cc <= NC; ++cc) J[r][cc] -= fct * J[k][cc];
            }
        }
#pragma unroll
        for (int k = NC - 1; k >= 0; --k) {
            T s = J[k][NC];
#pragma unroll
            for (int cc = k + 1; cc < NC; ++cc) s -= J[k][cc] * t1[cc];
            t1[k] = s * ip[k];
        }
        T smax = 0, xmax = 0;
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            x[a] += t1[a];
            smax = fmax(smax, fabs(t1[a]));
            xmax = fmax(xmax, fabs(x[a]));
        }
        if (smax <= tol * (T(1) + xmax)) break;
    }
    // recover kappa and mu
    lap(x, t1);
#pragma unroll
    for (int a = 0; a < NC; ++a) t1[a] = f3[a] + e * t1[a];
    lap(t1, t2);
#pragma unroll
    for (int a = 0; a < NC; ++a) {
        ka[a] = t1[a];
        mu[a] = f2[a] + nl_value<T, (Op::XK ? 2 : 1), Op::PB>(x[a], pbv[a], xkv[a]) + alv[a] * x[a] + t2[a];
        phi[a] = x[a];
    }
}

// Coarsest grid, Poisson: w = G f + mean(v) (the mean of w is free; keep the
// correction mean-free).  One thread per cell.
template <typename T>
__device__ void coarse_solve_poisson(T* w, const T* f, const T* v, const double* G, int ncell) {
    const int t = threadIdx.x;
    __shared__ T mv;
    if (t == 0) {
        T s = 0;
        for (int k = 0; k < ncell; ++k) s += v[k];
        mv = s / T(ncell);
    }
    __syncthreads();
    if (t < ncell) {
        T s = 0;
        for (int k = 0; k < ncell; ++k) s += (T)G[t * ncell + k] * f[k];
        w[t] = s + mv;
    }
}

template <class Op, int NTP, int NC, bool NEU>
__device__ __forceinline__ void coarse_body(const Op& op_top,
                                            const CoarseArgs<typename Op::real>& A,
                                            const CycleState* stop);

template <class Op, int NTP, int NC, bool NEU>
__global__ void __launch_bounds__(NTP) k_coarse_persistent(Op op_top, CoarseArgs<typename Op::real> A,
                                                           const CycleState* stop) {
    coarse_body<Op, NTP, NC, NEU>(op_top, A, stop);
}

// Batched: workgroup b runs the coarse levels of grid b.
template <class Op>
struct BatchCoarse {
    Op op;
    CoarseArgs<typename Op::real> A;
    const CycleState* stop;
};

template <class Op, int NTP, int NC, bool NEU>
__global__ void __launch_bounds__(NTP) k_coarse_persistent_batched(
    const BatchCoarse<Op>* __restrict__ args) {
    const BatchCoarse<Op>& B = args[blockIdx.x];
    coarse_body<Op, NTP, NC, NEU>(B.op, B.A, B.stop);
}

template <class Op, int NTP, int NC, bool NEU>
__device__ __forceinline__ void coarse_body(const Op& op_top,
                                            const CoarseArgs<typename Op::real>& A,
                                            const CycleState* stop) {
    using T = typename Op::real;
    constexpr int NF = Op::NF;
    __shared__ T Su[NF][CP_TOTAL];
    __shared__ T Sf[NF][CP_TOTAL];
    __shared__ T Sv[NF][CP_TOTAL];
    __shared__ T Sxk[Op::XK ? CP_TOTAL : 1];
    __shared__ T Spb[Op::PB ? CP_TOTAL : 1];
    __shared__ T Spw[Op::PW ? CP_TOTAL : 1];
    if (stopped(stop)) return;
    const int t = threadIdx.x;
    const CoarseGeom& G = A.geo;
    const int N0 = G.m[0] * G.n[0];
    // load the top level: every stride's loads are issued before the LDS
    // stores (indices clamped to the last cell, which is then stored twice
    // with the same value)
    {
        constexpr int NQ = (CP_CELLS + NTP - 1) / NTP;
        constexpr int NV = 2 * NF + (Op::XK ? 1 : 0) + (Op::PB ? 1 : 0) + (Op::PW ? 1 : 0);
        T v[NQ][NV];
        int qs[NQ];
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            const int q = min(t + j * NTP, N0 - 1);
            qs[j] = q;
            int k = 0;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                v[j][k++] = A.u[f][q];
                v[j][k++] = A.rr[f][q];
            }
            if constexpr (Op::XK) v[j][k++] = A.xk[q];
            if constexpr (Op::PB) v[j][k++] = A.pb[q];
            if constexpr (Op::PW) v[j][k++] = A.pin[q];
        }
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            const int q = qs[j];
            int k = 0;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                Su[f][q] = v[j][k++];
                Sf[f][q] = v[j][k++];
            }
            if constexpr (Op::XK) Sxk[q] = v[j][k++];
            if constexpr (Op::PB) Spb[q] = v[j][k++];
            if constexpr (Op::PW) Spw[q] = v[j][k++];
        }
    }
    __syncthreads();
    // coefficient pyramids (2x2 averages)
    if constexpr (Op::XK || Op::PB || Op::PW) {
        for (int l = 1; l < G.nlev; ++l) {
            const int mf = G.m[l - 1], lmc = G.lm[l], mcv = G.m[l];
            for (int q = t; q < mcv * G.n[l]; q += NTP) {
                const int I = q & (mcv - 1), J = q >> lmc;
                const int a = G.off[l - 1] + 2 * J * mf + 2 * I;
                if constexpr (Op::XK)
                    Sxk[G.off[l] + q] = T(0.25) * ((Sxk[a] + Sxk[a + 1]) + (Sxk[a + mf] + Sxk[a + mf + 1]));
                if constexpr (Op::PB)
                    Spb[G.off[l] + q] = T(0.25) * ((Spb[a] + Spb[a + 1]) + (Spb[a + mf] + Spb[a + mf + 1]));
                if constexpr (Op::PW)
                    Spw[G.off[l] + q] = T(0.25) * ((Spw[a] + Spw[a + 1]) + (Spw[a + mf] + Spw[a + mf + 1]));
            }
            __syncthreads();
        }
    }
    // level l has spacing 2^l h_top: scale 1/h^2 (and h^2) by exact powers of two
    auto opl = [&](int l) {
        Op o = op_top;
        if constexpr (NF == 3) o.op.ih2 = ldexp(op_top.op.ih2, -2 * l);
        else { o.ih2 = ldexp(op_top.ih2, -2 * l); o.h2 = ldexp(op_top.h2, 2 * l); }
        return o;
    };
    // sum of the four neighbours (ghost rule of each axis) of cell (i, j) of
    // an m x n level
    const bool nbx = G.bc & BC_NEUMANN_X, nby = G.bc & BC_NEUMANN_Y;
    auto nsum_l = [&](const T* a, int i, int j, int m, int lm, int n) {
        const int r = j << lm;
        return (a[bidx<NEU>(i + 1, m, nbx) + r] + a[bidx<NEU>(i - 1, m, nbx) + r]) +
               (a[i + (bidx<NEU>(j + 1, n, nby) << lm)] + a[i + (bidx<NEU>(j - 1, n, nby) << lm)]);
    };
    auto complete_rhs = [&](int l) {
        const Op o = opl(l);
        const int m = G.m[l], lm = G.lm[l], n = G.n[l], off = G.off[l];
        for (int q = t; q < m * n; q += NTP) {
            const int i = q & (m - 1), j = q >> lm;
            T u[NF], ns[NF], N[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) { u[f] = Su[f][off + q]; ns[f] = nsum_l(&Su[f][off], i, j, m, lm, n); }
            o.apply(u, ns, Op::XK ? Sxk[off + q] : T(0), Op::PB ? Spb[off + q] : T(0),
                    Op::PW ? Spw[off + q] : T(0), N);
#pragma unroll
            for (int f = 0; f < NF; ++f) Sf[f][off + q] += N[f];
        }
        __syncthreads();
    };
    auto sweeps = [&](int l, int nsw) {
        const Op o = opl(l);
        const int m = G.m[l], lm = G.lm[l], n = G.n[l], off = G.off[l];
        for (int p = 0; p < nsw; ++p) {
            const int colour = p & 1;
            for (int q2 = t; q2 < (m * n) >> 1; q2 += NTP) {
                const int j = q2 >> (lm - 1), k = q2 & ((m >> 1) - 1);
                const int i = 2 * k + ((j + colour) & 1);
                const int q = (j << lm) + i;
                T u[NF], ns[NF], fv[NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    u[f] = Su[f][off + q];
                    ns[f] = nsum_l(&Su[f][off], i, j, m, lm, n);
                    fv[f] = Sf[f][off + q];
                }
                o.relax(u, ns, fv, Op::XK ? Sxk[off + q] : T(0), Op::PB ? Spb[off + q] : T(0),
                        Op::PW ? Spw[off + q] : T(0));
#pragma unroll
                for (int f = 0; f < NF; ++f) Su[f][off + q] = u[f];
            }
            __syncthreads();
        }
    };
    const int L = G.nlev;
    // down
    if (A.complete_top) complete_rhs(0);
    for (int l = 0; l < L - 1; ++l) {
        sweeps(l, A.nsw1);
        const Op o = opl(l);
        const int m = G.m[l], lm = G.lm[l], n = G.n[l], off = G.off[l];
        const int mc = G.m[l + 1], lmc = G.lm[l + 1], nc = G.n[l + 1], offc = G.off[l + 1];
        for (int Q = t; Q < mc * nc; Q += NTP) {
            const int I = Q & (mc - 1), J = Q >> lmc;
            T su[NF], sr[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) { su[f] = T(0); sr[f] = T(0); }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int i = 2 * I + (c & 1), j = 2 * J + (c >> 1);
                const int q = (j << lm) + i;
                T u[NF], ns[NF], N[NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) { u[f] = Su[f][off + q]; ns[f] = nsum_l(&Su[f][off], i, j, m, lm, n); }
                o.apply(u, ns, Op::XK ? Sxk[off + q] : T(0), Op::PB ? Spb[off + q] : T(0),
                    Op::PW ? Spw[off + q] : T(0), N);
#pragma unroll
                for (int f = 0; f < NF; ++f) { su[f] += u[f]; sr[f] += Sf[f][off + q] - N[f]; }
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                Su[f][offc + Q] = T(0.25) * su[f];
                Sv[f][offc + Q] = T(0.25) * su[f];
                Sf[f][offc + Q] = T(0.25) * sr[f];
            }
        }
        __syncthreads();
        complete_rhs(l + 1);
    }
    // coarsest
    {
        const int l = L - 1, off = G.off[l], nc = G.m[l] * G.n[l];
        if constexpr (NF == 3) {
            // the host launches the instantiation whose NC equals the coarsest cell count
            if (t == 0 && nc == NC) {
                const Op o = opl(l);
                T fbuf[3 * NC];
#pragma unroll
                for (int q = 0; q < NC; ++q) {
                    fbuf[q] = Sf[0][off + q];
                    fbuf[NC + q] = Sf[1][off + q];
                    fbuf[2 * NC + q] = Sf[2][off + q];
                }
                T* xkp = Op::XK ? &Sxk[off] : nullptr;
                T* pbp = Op::PB ? &Spb[off] : nullptr;
                T* pwp = Op::PW ? &Spw[off] : nullptr;
                coarse_solve_mpfc<Op, NC>(o, &Su[0][off], &Su[1][off], &Su[2][off], fbuf, xkp, pbp, pwp,
                                          G.m[l], G.lm[l], G.n[l], NEU ? G.bc : 0,
                                          A.newton_maxit, A.newton_tol);
            }
        } else {
            coarse_solve_poisson<T>(&Su[0][off], &Sf[0][off], &Sv[0][off], A.G, nc);
        }
        __syncthreads();
    }
    // up
    for (int l = L - 2; l >= 0; --l) {
        const int m = G.m[l], lm = G.lm[l], n = G.n[l], off = G.off[l];
        const int mc = G.m[l + 1], nc = G.n[l + 1], offc = G.off[l + 1];
        for (int q = t; q < m * n; q += NTP) {
            const int i = q & (m - 1), j = q >> lm, I = i >> 1, J = j >> 1;
            const int Is = bidx<NEU>((i & 1) ? I + 1 : I - 1, mc, nbx);
            const int Js = bidx<NEU>((j & 1) ? J + 1 : J - 1, nc, nby);
#pragma unroll
            for (int f = 0; f < NF; ++f)
                Su[f][off + q] += bilinear<T>(&Su[f][offc], &Sv[f][offc], I, J, Is, Js, mc);
        }
        __syncthreads();
        sweeps(l, A.nsw2);
    }
    // top level back to global memory
    for (int q = t; q < N0; q += NTP) {
#pragma unroll
        for (int f = 0; f < NF; ++f) A.u[f][q] = Su[f][q];
    }
}

// ---------------------------------------------------------------------------
// Coarsest level of a grid whose sides are not all powers of two.  Such a grid
// is coarsened while both sides of the next level stay even, so its coarsest
// level (m x n, both even, at most CG_CELLS cells; 64 x 50 for 512 x 400) can
// be far larger than the 2 x 2 grid the dense Newton solve is made for.  One
// workgroup of CG_THREADS threads; every index is general (no power-of-two
// masks), and each axis follows its ghost rule.
constexpr int CG_THREADS = 1024;
constexpr int CG_CELLS = 4096;
constexpr int CG_SLOTS = CG_CELLS / 2 / CG_THREADS;  // cells of one colour per thread

// MPFC system: complete the FAS right-hand side f = R r + N(u), then relax the
// level by A.nsw2 half-sweeps of the red-black collective smoother (the
// coarsest "solve" is approximate; the finer levels correct what it leaves).
// u lives in LDS; f and the coefficients of each thread's cells in registers.
template <class Op, bool NEU>
__global__ void __launch_bounds__(CG_THREADS) k_coarsest_sweeps(Op op,
                                                                CoarseArgs<typename Op::real> A,
                                                                const CycleState* stop) {
    using T = typename Op::real;
    constexpr int NF = Op::NF;
    __shared__ T Su[NF][CG_CELLS];
    if (stopped(stop)) return;
    const int t = threadIdx.x;
    const int m = A.geo.m[0], n = A.geo.n[0], N = m * n, mh = m >> 1;
    const bool nbx = NEU && (A.geo.bc & BC_NEUMANN_X), nby = NEU && (A.geo.bc & BC_NEUMANN_Y);
    for (int q = t; q < N; q += CG_THREADS) {
#pragma unroll
        for (int f = 0; f < NF; ++f) Su[f][q] = A.u[f][q];
    }
    __syncthreads();
    auto nsum = [&](const T* a, int i, int j) {
        const int ie = i + 1 < m ? i + 1 : (nbx ? m - 1 : 0);
        const int iw = i > 0 ? i - 1 : (nbx ? 0 : m - 1);
        const int jn = j + 1 < n ? j + 1 : (nby ? n - 1 : 0);
        const int js = j > 0 ? j - 1 : (nby ? 0 : n - 1);
        const int r = j * m;
        return (a[ie + r] + a[iw + r]) + (a[i + jn * m] + a[i + js * m]);
    };
    // slot s of colour c of this thread: cell (i, j), or q = -1 for none
    auto cell = [&](int c, int s, int& i, int& j) {
        const int q2 = t + s * CG_THREADS;
        if (q2 >= (N >> 1)) return -1;
        j = q2 / mh;
        i = 2 * (q2 - j * mh) + ((j + c) & 1);
        return j * m + i;
    };
    T fr[2][CG_SLOTS][NF], xkr[2][CG_SLOTS], pbr[2][CG_SLOTS], wr[2][CG_SLOTS];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
#pragma unroll
        for (int s = 0; s < CG_SLOTS; ++s) {
#pragma unroll
            for (int f = 0; f < NF; ++f) fr[c][s][f] = T(0);
            xkr[c][s] = T(0);
            pbr[c][s] = T(0);
            wr[c][s] = T(0);
            int i = 0, j = 0;
            const int q = cell(c, s, i, j);
            if (q < 0) continue;
            if constexpr (Op::XK) xkr[c][s] = A.xk[q];
            if constexpr (Op::PB) pbr[c][s] = A.pb[q];
            if constexpr (Op::PW) wr[c][s] = A.pin[q];
            T u[NF], ns[NF], Nu[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                u[f] = Su[f][q];
                ns[f] = nsum(Su[f], i, j);
                fr[c][s][f] = A.rr[f][q];
            }
            if (A.complete_top) {
                op.apply(u, ns, xkr[c][s], pbr[c][s], wr[c][s], Nu);
#pragma unroll
                for (int f = 0; f < NF; ++f) fr[c][s][f] += Nu[f];
            }
        }
    }
    __syncthreads();  // every N(u) above read u as loaded
    auto pass = [&](auto colc) {
        constexpr int c = decltype(colc)::value;
#pragma unroll
        for (int s = 0; s < CG_SLOTS; ++s) {
            int i = 0, j = 0;
            const int q = cell(c, s, i, j);
            if (q < 0) continue;
            T u[NF], ns[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                u[f] = Su[f][q];
                ns[f] = nsum(Su[f], i, j);
            }
            op.relax(u, ns, fr[c][s], xkr[c][s], pbr[c][s], wr[c][s]);
#pragma unroll
            for (int f = 0; f < NF; ++f) Su[f][q] = u[f];
        }
    };
    for (int p = 0; p < A.nsw2; ++p) {
        if ((p & 1) == 0) pass(std::integral_constant<int, 0>{});
        else pass(std::integral_constant<int, 1>{});
        __syncthreads();
    }
    for (int q = t; q < N; q += CG_THREADS) {
#pragma unroll
        for (int f = 0; f < NF; ++f) A.u[f][q] = Su[f][q];
    }
}

// Poisson problem -Lap_h w = f on the same coarsest level, solved exactly in
// the separable eigenbasis of the operator: with V_x (m x m) and V_y (n x n)
// the orthonormal eigenvectors of the one-dimensional second difference under
// each axis' boundary rule (columns: modes) and lam the eigenvalue sums,
//   w = V_y [ (V_y^T F V_x) / lam ] V_x^T + mean(v),
// the (0, 0) mode dropped (1/lam stored as 0), F the m x n grid function f.
// A.G holds V_x (row i: cell, column k: mode), then V_y, then 1/lam (row l:
// y mode, column k: x mode).  v is u as loaded (the restricted iterate): the
// correction keeps mean zero, as the dense Green's-matrix solve does.
template <typename T>
__global__ void __launch_bounds__(CG_THREADS) k_coarsest_poisson(PoissonOp<T> op, CoarseArgs<T> A,
                                                                 const CycleState* stop) {
    __shared__ T S0[CG_CELLS];
    __shared__ T S1[CG_CELLS];
    __shared__ double red[CG_THREADS / 64];
    __shared__ double mean_v;
    if (stopped(stop)) return;
    const int t = threadIdx.x;
    const int m = A.geo.m[0], n = A.geo.n[0], N = m * n;
    const bool nbx = A.geo.bc & BC_NEUMANN_X, nby = A.geo.bc & BC_NEUMANN_Y;
    const double* Vx = A.G;
    const double* Vy = Vx + (size_t)m * m;
    const double* il = Vy + (size_t)n * n;
    double sv = 0.0;
    for (int q = t; q < N; q += CG_THREADS) {
        S0[q] = A.u[0][q];
        sv += (double)S0[q];
    }
    const double tot = block_sum<CG_THREADS>(sv, red);  // contains a barrier
    if (t == 0) mean_v = tot / (double)N;
    for (int q = t; q < N; q += CG_THREADS) {
        const int j = q / m, i = q - j * m;
        const int ie = i + 1 < m ? i + 1 : (nbx ? m - 1 : 0);
        const int iw = i > 0 ? i - 1 : (nbx ? 0 : m - 1);
        const int jn = j + 1 < n ? j + 1 : (nby ? n - 1 : 0);
        const int js = j > 0 ? j - 1 : (nby ? 0 : n - 1);
        T f = A.rr[0][q];
        if (A.complete_top) {
            const T u[1] = {S0[q]};
            const T ns[1] = {(S0[ie + j * m] + S0[iw + j * m]) + (S0[i + jn * m] + S0[i + js * m])};
            T Nu[1];
            op.apply(u, ns, T(0), T(0), T(0), Nu);
            f += Nu[0];
        }
        S1[q] = f;
    }
    __syncthreads();
    // S0 = F V_x   (row j, column k)
    for (int q = t; q < N; q += CG_THREADS) {
        const int j = q / m, k = q - j * m;
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += (double)S1[j * m + i] * Vx[(size_t)i * m + k];
        S0[q] = (T)s;
    }
    __syncthreads();
    // S1 = (V_y^T S0) / lam   (row l, column k)
    for (int q = t; q < N; q += CG_THREADS) {
        const int l = q / m, k = q - l * m;
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += Vy[(size_t)j * n + l] * (double)S0[j * m + k];
        S1[q] = (T)(s * il[q]);
    }
    __syncthreads();
    // S0 = V_y S1   (row j, column k)
    for (int q = t; q < N; q += CG_THREADS) {
        const int j = q / m, k = q - j * m;
        double s = 0.0;
        for (int l = 0; l < n; ++l) s += Vy[(size_t)j * n + l] * (double)S1[l * m + k];
        S0[q] = (T)s;
    }
    __syncthreads();
    // w = S0 V_x^T + mean(v)
    const double mv = mean_v;
    for (int q = t; q < N; q += CG_THREADS) {
        const int j = q / m, i = q - j * m;
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += (double)S0[j * m + k] * Vx[(size_t)i * m + k];
        A.u[0][q] = (T)(s + mv);
    }
}

}  // namespace mpfc
