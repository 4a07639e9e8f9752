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
//
// Storage inside the solver is split by colour: a level of N cells holds its
// red cells ((i + j + k) even) in the first N/2 entries and its black cells in
// the last N/2, each half in (k, j, i/2) order (sidx).  A half-sweep then reads
// and writes its own colour contiguously and reads the other colour as
// neighbours, so no cache line is fetched or written back for half of its
// bytes.  The caller's arrays stay in natural order (at3); the per-step
// kernels convert on the way in and out.  Workgroups take their cells in
// XCD-contiguous order (xcd_item), so the neighbouring rows and planes a
// workgroup reads are mostly in its own XCD's L2.
#pragma once
#include "step.hpp"
#include "tiles.hpp"

namespace mpfc {

struct Grid3 {
    int m, n, l;      // cells along x, y, z (powers of two)
    int lm, ln, ll;   // their log2
};

// Natural index (the caller's arrays).
__device__ __forceinline__ size_t at3(int i, int j, int k, const Grid3& g) {
    return ((((size_t)k << g.ln) + (size_t)j) << g.lm) + (size_t)i;
}
__device__ __forceinline__ size_t cells3(const Grid3& g) { return (size_t)g.m * g.n * g.l; }
// Colour-split index (the solver's arrays).
__device__ __forceinline__ size_t sidx(int i, int j, int k, const Grid3& g) {
    const size_t half = cells3(g) >> 1;
    return (((i + j + k) & 1) ? half : 0) + ((((size_t)k << g.ln) + (size_t)j) << (g.lm - 1)) +
           (size_t)(i >> 1);
}
// Cell (i, j, k) of colour-split entry t.
__device__ __forceinline__ void split_cell(size_t t, const Grid3& g, int& i, int& j, int& k) {
    const size_t half = cells3(g) >> 1;
    const int c = t >= half ? 1 : 0;
    const size_t r = t - (c ? half : 0);
    const int ii = (int)(r & (size_t)((g.m >> 1) - 1));
    const size_t row = r >> (g.lm - 1);
    j = (int)(row & (size_t)(g.n - 1));
    k = (int)(row >> g.ln);
    i = 2 * ii + ((j + k + c) & 1);
}
// Entry handled by thread `threadIdx.x` of workgroup blockIdx.x, blocks dealt
// XCD-contiguously.
__device__ __forceinline__ size_t item3() {
    return (size_t)xcd_item(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
}

// Sum of the six face neighbours (periodic wrap-around), colour-split storage.
__device__ __forceinline__ double nsum6(const double* __restrict__ f, int i, int j, int k,
                                        const Grid3& g) {
    const int ip = (i + 1) & (g.m - 1), im = (i - 1) & (g.m - 1);
    const int jp = (j + 1) & (g.n - 1), jm = (j - 1) & (g.n - 1);
    const int kp = (k + 1) & (g.l - 1), km = (k - 1) & (g.l - 1);
    return ((f[sidx(ip, j, k, g)] + f[sidx(im, j, k, g)]) + (f[sidx(i, jp, k, g)] + f[sidx(i, jm, k, g)])) +
           (f[sidx(i, j, kp, g)] + f[sidx(i, j, km, g)]);
}
// The same in natural storage.
__device__ __forceinline__ double nsum6n(const double* __restrict__ f, int i, int j, int k,
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
    const size_t half = cells3(g) >> 1;
    const size_t t = item3();
    if (t >= half) return;
    int i, j, k;
    const size_t q = (colour ? half : 0) + t;
    split_cell(q, g, i, j, k);
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
// One thread per coarse cell, in natural coarse order: the two fine cells of a
// coarse cell along x (one per colour) sit at the same offset of the two
// halves, so consecutive threads read consecutive fine entries.  g is the fine
// grid.
template <class Op>
__global__ void __launch_bounds__(256) k3_restrict(Op op, Grid3 g, L3 A, L3 H, double* vH0,
                                                   double* vH1, double* vH2, double* rH0,
                                                   double* rH1, double* rH2, double* xkH,
                                                   const CycleState* st) {
    if (stopped(st)) return;
    const Grid3 c{g.m >> 1, g.n >> 1, g.l >> 1, g.lm - 1, g.ln - 1, g.ll - 1};
    const size_t Qn = item3();
    if (Qn >= cells3(c)) return;
    const int I = (int)(Qn & (size_t)(c.m - 1));
    const int J = (int)((Qn >> c.lm) & (size_t)(c.n - 1));
    const int K = (int)(Qn >> (c.lm + c.ln));
    const size_t Q = sidx(I, J, K, c);
    constexpr int NF = Op::NF;
    double su[NF], sr[NF], sxk = 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f) { su[f] = 0.0; sr[f] = 0.0; }
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
        const int i = 2 * I + (cc & 1), j = 2 * J + ((cc >> 1) & 1), k = 2 * K + (cc >> 2);
        const size_t q = sidx(i, j, k, g);
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
    const size_t q = item3();
    if (q >= cells3(g)) return;
    int i, j, k;
    split_cell(q, g, i, j, k);
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

// Coarse correction in place: vH = uH - vH (vH is not needed afterwards), so
// the prolongation reads one array per field.  g is the coarse grid.
template <int NF>
__global__ void __launch_bounds__(256) k3_correction(Grid3 g, L3 H, double* vH0, double* vH1,
                                                     double* vH2, const CycleState* st) {
    if (stopped(st)) return;
    const size_t q = item3();
    if (q >= cells3(g)) return;
    double* vH[3] = {vH0, vH1, vH2};
#pragma unroll
    for (int f = 0; f < NF; ++f) vH[f][q] = H.u[f][q] - vH[f][q];
}

// u += trilinear interpolation of the coarse correction E = uH - vH (held in
// vH by k3_correction): per axis 3/4 of the parent's
// coarse index and 1/4 of the coarse neighbour on the fine cell's side.  One
// thread per pair of fine cells (2I, j, k), (2I + 1, j, k): they share the
// coarse parent, sit at the same offset of the two colour halves (so a wave
// reads and writes both halves contiguously) and need 12 coarse values
// between them.  g is the fine grid.
template <int NF>
__global__ void __launch_bounds__(256) k3_prolong(Grid3 g, L3 A, const double* E0,
                                                  const double* E1, const double* E2,
                                                  const CycleState* st) {
    if (stopped(st)) return;
    const size_t t = item3();
    if (t >= (cells3(g) >> 1)) return;
    const int I = (int)(t & (size_t)((g.m >> 1) - 1));
    const size_t row = t >> (g.lm - 1);
    const int j = (int)(row & (size_t)(g.n - 1)), k = (int)(row >> g.ln);
    const Grid3 c{g.m >> 1, g.n >> 1, g.l >> 1, g.lm - 1, g.ln - 1, g.ll - 1};
    // x: coarse I - 1, I, I + 1 (fine 2I takes I - 1 as its side, 2I + 1 takes I + 1)
    const int X[3] = {(I - 1) & (c.m - 1), I, (I + 1) & (c.m - 1)};
    const int Y[2] = {j >> 1, ((j >> 1) + ((j & 1) ? 1 : -1)) & (c.n - 1)};
    const int Z[2] = {k >> 1, ((k >> 1) + ((k & 1) ? 1 : -1)) & (c.l - 1)};
    const double w[2] = {0.75, 0.25};
    const double* E[3] = {E0, E1, E2};
    const size_t q0 = sidx(2 * I, j, k, g), q1 = sidx(2 * I + 1, j, k, g);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        double e[2][2][3];
#pragma unroll
        for (int z = 0; z < 2; ++z)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    e[z][y][x] = E[f][sidx(X[x], Y[y], Z[z], c)];
                }
        // fine 2I: parent X[1], side X[0]; fine 2I + 1: parent X[1], side X[2]
        double v0 = 0.0, v1 = 0.0;
#pragma unroll
        for (int z = 0; z < 2; ++z)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int x = 0; x < 2; ++x) {
                    v0 += w[x] * w[y] * w[z] * e[z][y][x == 0 ? 1 : 0];
                    v1 += w[x] * w[y] * w[z] * e[z][y][x == 0 ? 1 : 2];
                }
        A.u[f][q0] += v0;
        A.u[f][q1] += v1;
    }
}

// The same prolongation with the coarse correction staged in LDS, for fine
// grids with m >= 32 (n, l >= 4 hold on every fine level): a workgroup takes
// P3X x-pairs x P3Y rows x P3Z planes, whose coarse footprint (one coarse cell
// of margin on each side) is read from global memory once instead of twelve
// times per pair.  Same values, same order of operations as k3_prolong.
constexpr int P3X = 16, P3Y = 4, P3Z = 4;
template <int NF>
__global__ void __launch_bounds__(256) k3_prolong_blk(Grid3 g, L3 A, const double* E0,
                                                      const double* E1, const double* E2,
                                                      const CycleState* st) {
    static_assert(P3X * P3Y * P3Z == 256, "one x-pair per thread");
    constexpr int CXN = P3X + 2, CYN = P3Y / 2 + 2, CZN = P3Z / 2 + 2;
    __shared__ double Es[NF][CZN][CYN][CXN];
    if (stopped(st)) return;
    const int nbx = (g.m >> 1) / P3X, nby = g.n / P3Y;
    const int b = xcd_item(blockIdx.x, gridDim.x);
    const int bx = b % nbx, r = b / nbx, by = r % nby, bz = r / nby;
    const int I0 = bx * P3X, j0 = by * P3Y, k0 = bz * P3Z;
    const Grid3 c{g.m >> 1, g.n >> 1, g.l >> 1, g.lm - 1, g.ln - 1, g.ll - 1};
    const int cx0 = I0 - 1, cy0 = (j0 >> 1) - 1, cz0 = (k0 >> 1) - 1;
    const double* E[3] = {E0, E1, E2};
    for (int q = threadIdx.x; q < CXN * CYN * CZN; q += 256) {
        const int x = q % CXN, yz = q / CXN, y = yz % CYN, z = yz / CYN;
        const size_t Q = sidx((cx0 + x) & (c.m - 1), (cy0 + y) & (c.n - 1), (cz0 + z) & (c.l - 1), c);
#pragma unroll
        for (int f = 0; f < NF; ++f) Es[f][z][y][x] = E[f][Q];
    }
    __syncthreads();
    const int tx = threadIdx.x & (P3X - 1), ty = (threadIdx.x / P3X) & (P3Y - 1),
              tz = threadIdx.x / (P3X * P3Y);
    const int I = I0 + tx, j = j0 + ty, k = k0 + tz;
    // local coarse indices: parent x tx + 1 with sides tx, tx + 2; parent y
    // (ty >> 1) + 1 with its side on the fine cell's side; z alike
    const int LY[2] = {(ty >> 1) + 1, (ty >> 1) + 1 + ((j & 1) ? 1 : -1)};
    const int LZ[2] = {(tz >> 1) + 1, (tz >> 1) + 1 + ((k & 1) ? 1 : -1)};
    const double w[2] = {0.75, 0.25};
    const size_t q0 = sidx(2 * I, j, k, g), q1 = sidx(2 * I + 1, j, k, g);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        double e[2][2][3];
#pragma unroll
        for (int z = 0; z < 2; ++z)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int x = 0; x < 3; ++x) e[z][y][x] = Es[f][LZ[z]][LY[y]][tx + x];
        double v0 = 0.0, v1 = 0.0;
#pragma unroll
        for (int z = 0; z < 2; ++z)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int x = 0; x < 2; ++x) {
                    v0 += w[x] * w[y] * w[z] * e[z][y][x == 0 ? 1 : 0];
                    v1 += w[x] * w[y] * w[z] * e[z][y][x == 0 ? 1 : 2];
                }
        A.u[f][q0] += v0;
        A.u[f][q1] += v1;
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
    // each workgroup sums one contiguous range (XCD-contiguous order)
    const size_t chunk = ((total + gridDim.x - 1) / gridDim.x + NT - 1) / NT * NT;
    const size_t b0 = (size_t)xcd_item(blockIdx.x, gridDim.x) * chunk;
    const size_t b1 = b0 + chunk < total ? b0 + chunk : total;
    for (size_t q = b0 + threadIdx.x; q < b1; q += NT) {
        int i, j, k;
        split_cell(q, g, i, j, k);
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

// ---- levels of at most CP3_CELLS cells: one persistent workgroup ---------------
// The small levels of a V-cycle are latency bound (a launch each for every
// half-sweep, restriction, completion and prolongation).  This kernel runs
// them all, from the first level of at most CP3_CELLS cells down to the
// coarsest and back, in LDS (natural order inside), with the same arithmetic
// as the per-level kernels: complete the top level's right-hand side, nu1
// half-sweep pairs, restriction with completion, coarsest sweeps, trilinear
// correction, nu2 pairs; the top level's u returns to global memory.
constexpr int CP3_CELLS = 512;
constexpr int CP3_TOTAL = 640;    // all levels below 512 cells: 512 + 64 + 8 (+ padding)
constexpr int CP3_MAXLEV = 10;
constexpr int CP3_THREADS = 256;

struct CoarseGeom3 {
    int nlev;
    int m[CP3_MAXLEV], n[CP3_MAXLEV], l[CP3_MAXLEV];
    int lm[CP3_MAXLEV], ln[CP3_MAXLEV];
    int off[CP3_MAXLEV];
};

struct CoarseArgs3 {
    CoarseGeom3 geo;
    Grid3 gtop;            // top level (its global arrays are colour-split)
    double* u[3];          // top level u (in/out)
    const double* f[3];    // top level R r (complete_top = 1) or complete right-hand side
    const double* xk;      // top level phi^k (scheme 2)
    int complete_top;
    int nsw1, nsw2, nswc;  // half-sweep pairs down / up / on the coarsest level
};

__device__ __forceinline__ MpfcOp3<1, true> op_level(MpfcOp3<1, true> o, int l) { o.op.ih2 = ldexp(o.op.ih2, -2 * l); return o; }
__device__ __forceinline__ MpfcOp3<1, false> op_level(MpfcOp3<1, false> o, int l) { o.op.ih2 = ldexp(o.op.ih2, -2 * l); return o; }
__device__ __forceinline__ MpfcOp3<2, true> op_level(MpfcOp3<2, true> o, int l) { o.op.ih2 = ldexp(o.op.ih2, -2 * l); return o; }
__device__ __forceinline__ MpfcOp3<2, false> op_level(MpfcOp3<2, false> o, int l) { o.op.ih2 = ldexp(o.op.ih2, -2 * l); return o; }
__device__ __forceinline__ PoissonOp3 op_level(PoissonOp3 o, int l) {
    o.ih2 = ldexp(o.ih2, -2 * l);
    o.h2 = ldexp(o.h2, 2 * l);
    return o;
}

template <class Op>
__global__ void __launch_bounds__(CP3_THREADS) k3_coarse(Op op_top, CoarseArgs3 A,
                                                         const CycleState* st) {
    constexpr int NF = Op::NF;
    constexpr int NT = CP3_THREADS;
    __shared__ double Su[NF][CP3_TOTAL];
    __shared__ double Sf[NF][CP3_TOTAL];
    __shared__ double Sv[NF][CP3_TOTAL];
    __shared__ double Sx[Op::XK ? CP3_TOTAL : 1];
    if (stopped(st)) return;
    const int t = threadIdx.x;
    const CoarseGeom3& G = A.geo;
    const int L = G.nlev;
    auto dec = [&](int l, int q, int& i, int& j, int& k) {
        i = q & (G.m[l] - 1);
        j = (q >> G.lm[l]) & (G.n[l] - 1);
        k = q >> (G.lm[l] + G.ln[l]);
    };
    auto nat = [&](int l, int i, int j, int k) { return (((k << G.ln[l]) + j) << G.lm[l]) + i; };
    auto ns6 = [&](const double* a, int l, int i, int j, int k) {
        const int ip = (i + 1) & (G.m[l] - 1), im = (i - 1) & (G.m[l] - 1);
        const int jp = (j + 1) & (G.n[l] - 1), jm = (j - 1) & (G.n[l] - 1);
        const int kp = (k + 1) & (G.l[l] - 1), km = (k - 1) & (G.l[l] - 1);
        return ((a[nat(l, ip, j, k)] + a[nat(l, im, j, k)]) + (a[nat(l, i, jp, k)] + a[nat(l, i, jm, k)])) +
               (a[nat(l, i, j, kp)] + a[nat(l, i, j, km)]);
    };
    auto cells = [&](int l) { return G.m[l] * G.n[l] * G.l[l]; };
    // load the top level (colour-split in global memory, natural here)
    const int N0 = cells(0);
    for (int q = t; q < N0; q += NT) {
        int i, j, k;
        split_cell((size_t)q, A.gtop, i, j, k);
        const int p = nat(0, i, j, k);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            Su[f][p] = A.u[f][q];
            Sf[f][p] = A.f[f][q];
        }
        if constexpr (Op::XK) Sx[p] = A.xk[q];
    }
    __syncthreads();
    auto complete = [&](int l) {
        const Op o = op_level(op_top, l);
        const int off = G.off[l];
        for (int q = t; q < cells(l); q += NT) {
            int i, j, k;
            dec(l, q, i, j, k);
            double u[NF], ns[NF], N[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                u[f] = Su[f][off + q];
                ns[f] = ns6(&Su[f][off], l, i, j, k);
            }
            o.apply(u, ns, Op::XK ? Sx[off + q] : 0.0, N);
#pragma unroll
            for (int f = 0; f < NF; ++f) Sf[f][off + q] += N[f];
        }
        __syncthreads();
    };
    auto sweeps = [&](int l, int pairs) {
        const Op o = op_level(op_top, l);
        const int off = G.off[l];
        for (int p = 0; p < 2 * pairs; ++p) {
            const int colour = p & 1;
            for (int q = t; q < cells(l); q += NT) {
                int i, j, k;
                dec(l, q, i, j, k);
                if (((i + j + k) & 1) != colour) continue;
                double u[NF], ns[NF], fv[NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    u[f] = Su[f][off + q];
                    ns[f] = ns6(&Su[f][off], l, i, j, k);
                    fv[f] = Sf[f][off + q];
                }
                o.relax(u, ns, fv, Op::XK ? Sx[off + q] : 0.0);
#pragma unroll
                for (int f = 0; f < NF; ++f) Su[f][off + q] = u[f];
            }
            __syncthreads();
        }
    };
    if (A.complete_top) complete(0);
    for (int l = 0; l < L - 1; ++l) {
        sweeps(l, A.nsw1);
        const Op o = op_level(op_top, l);
        const int off = G.off[l], offc = G.off[l + 1];
        for (int Q = t; Q < cells(l + 1); Q += NT) {
            int I, J, K;
            dec(l + 1, Q, I, J, K);
            double su[NF], sr[NF], sx = 0.0;
#pragma unroll
            for (int f = 0; f < NF; ++f) { su[f] = 0.0; sr[f] = 0.0; }
#pragma unroll
            for (int cc = 0; cc < 8; ++cc) {
                const int i = 2 * I + (cc & 1), j = 2 * J + ((cc >> 1) & 1), k = 2 * K + (cc >> 2);
                const int q = nat(l, i, j, k);
                double u[NF], ns[NF], N[NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    u[f] = Su[f][off + q];
                    ns[f] = ns6(&Su[f][off], l, i, j, k);
                }
                const double xk = Op::XK ? Sx[off + q] : 0.0;
                o.apply(u, ns, xk, N);
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    su[f] += u[f];
                    sr[f] += Sf[f][off + q] - N[f];
                }
                sx += xk;
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                Su[f][offc + Q] = 0.125 * su[f];
                Sv[f][offc + Q] = 0.125 * su[f];
                Sf[f][offc + Q] = 0.125 * sr[f];
            }
            if constexpr (Op::XK) Sx[offc + Q] = 0.125 * sx;
        }
        __syncthreads();
        complete(l + 1);
    }
    sweeps(L - 1, A.nswc);
    for (int l = L - 2; l >= 0; --l) {
        const int off = G.off[l], offc = G.off[l + 1];
        const double w[2] = {0.75, 0.25};
        for (int q = t; q < cells(l); q += NT) {
            int i, j, k;
            dec(l, q, i, j, k);
            const int I[2] = {i >> 1, ((i >> 1) + ((i & 1) ? 1 : -1)) & (G.m[l + 1] - 1)};
            const int J[2] = {j >> 1, ((j >> 1) + ((j & 1) ? 1 : -1)) & (G.n[l + 1] - 1)};
            const int K[2] = {k >> 1, ((k >> 1) + ((k & 1) ? 1 : -1)) & (G.l[l + 1] - 1)};
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                double v = 0.0;
#pragma unroll
                for (int z = 0; z < 2; ++z)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
#pragma unroll
                        for (int x = 0; x < 2; ++x) {
                            const int Q = offc + nat(l + 1, I[x], J[y], K[z]);
                            v += w[x] * w[y] * w[z] * (Su[f][Q] - Sv[f][Q]);
                        }
                Su[f][off + q] += v;
            }
        }
        __syncthreads();
        sweeps(l, A.nsw2);
    }
    for (int q = t; q < N0; q += NT) {
        int i, j, k;
        split_cell((size_t)q, A.gtop, i, j, k);
        const int p = nat(0, i, j, k);
#pragma unroll
        for (int f = 0; f < NF; ++f) A.u[f][q] = Su[f][p];
    }
}

// ---- per-step passes ----------------------------------------------------------
// Source S (App. B.1 / B.2) with the seven-point Laplacian, from the caller's
// (natural-order) fields into colour-split storage.
template <int SCHEME>
__global__ void __launch_bounds__(256) k3_source(Grid3 g, double ih2, double d, double alpha,
                                                 const double* __restrict__ phik,
                                                 const double* __restrict__ phikm1,
                                                 const double* __restrict__ psik, double* S1,
                                                 double* S2, double* S3) {
    const size_t q = item3();
    if (q >= cells3(g)) return;
    int i, j, k;
    split_cell(q, g, i, j, k);
    const size_t p = at3(i, j, k, g);
    const double x = phik[p];
    const double lk = (nsum6n(phik, i, j, k, g) - 6.0 * x) * ih2;
    S1[q] = x + d * psik[p];
    if constexpr (SCHEME == 1) {
        S2[q] = 2.0 * lk;
        S3[q] = 0.0;
    } else {
        // Lap of phi~ = (3 phi^k - phi^{k-1})/2 from the two Laplacians
        const double lm1 = (nsum6n(phikm1, i, j, k, g) - 6.0 * phikm1[p]) * ih2;
        S2[q] = 0.5 * alpha * x + 2.0 * (0.5 * (3.0 * lk - lm1));
        S3[q] = 0.5 * lk;
    }
}

// kappa = S3 + e Lap phi (completion of the guess, first half).
__global__ void __launch_bounds__(256) k3_complete_kappa(Grid3 g, double ih2, double e,
                                                         const double* __restrict__ phi,
                                                         const double* __restrict__ S3,
                                                         double* ka) {
    const size_t q = item3();
    if (q >= cells3(g)) return;
    int i, j, k;
    split_cell(q, g, i, j, k);
    ka[q] = S3[q] + e * ((nsum6(phi, i, j, k, g) - 6.0 * phi[q]) * ih2);
}

// mu = S2 + g(phi) + al phi + Lap kappa (second half).
template <int SCHEME>
__global__ void __launch_bounds__(256) k3_complete_mu(Grid3 g, double ih2, double al,
                                                      const double* __restrict__ phi,
                                                      const double* __restrict__ phik,
                                                      const double* __restrict__ S2,
                                                      const double* __restrict__ ka, double* mu) {
    const size_t q = item3();
    if (q >= cells3(g)) return;
    int i, j, k;
    split_cell(q, g, i, j, k);
    const double x = phi[q];
    mu[q] = S2[q] + nl_value<double, SCHEME, false>(x, 0.0, SCHEME == 2 ? phik[q] : 0.0) +
            al * x + (nsum6(ka, i, j, k, g) - 6.0 * ka[q]) * ih2;
}

// phi^(0) = phi^k (mode 0) or 2 phi^k - phi^{k-1} (mode 1), into split storage;
// the solver's copy of phi^k (xk, split) too.
__global__ void __launch_bounds__(256) k3_guess(Grid3 g, int mode, const double* __restrict__ phik,
                                                const double* __restrict__ phikm1, double* phi,
                                                double* xk) {
    const size_t q = item3();
    if (q >= cells3(g)) return;
    int i, j, k;
    split_cell(q, g, i, j, k);
    const size_t p = at3(i, j, k, g);
    phi[q] = mode == 1 ? 2.0 * phik[p] - phikm1[p] : phik[p];
    if (xk) xk[q] = phik[p];
}

// dst (natural order) = src (split storage).
__global__ void __launch_bounds__(256) k3_from_split(Grid3 g, const double* __restrict__ src,
                                                     double* dst) {
    const size_t q = item3();
    if (q >= cells3(g)) return;
    int i, j, k;
    split_cell(q, g, i, j, k);
    dst[at3(i, j, k, g)] = src[q];
}

// psi^{k+1} in place (eq. discrete_1_b / discrete_2_b) and phi^{k+1} out, both
// in natural order, from the solver's phi (split storage).
template <int SCHEME>
__global__ void __launch_bounds__(256) k3_psi_update(Grid3 g, double s,
                                                     const double* __restrict__ phi,
                                                     const double* __restrict__ phik, double* psi,
                                                     double* phi_out) {
    const size_t q = item3();
    if (q >= cells3(g)) return;
    int i, j, k;
    split_cell(q, g, i, j, k);
    const size_t p = at3(i, j, k, g);
    const double x = phi[q];
    if constexpr (SCHEME == 1) psi[p] = (x - phik[p]) / s;
    else psi[p] = (2.0 / s) * (x - phik[p]) - psi[p];
    phi_out[p] = x;
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
        int i, j, k;
        split_cell(q, g, i, j, k);
        const double v = psi[at3(i, j, k, g)] - mean;   // psi: natural; b, w: split
        b[q] = v;
        sb += v * v;
        if (w) {
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
        int i, j, k;
        split_cell(q, g, i, j, k);
        const size_t qe = at3((i + 1) & (g.m - 1), j, k, g);
        const size_t qn = at3(i, (j + 1) & (g.n - 1), k, g);
        const size_t qt = at3(i, j, (k + 1) & (g.l - 1), g);
        const size_t p = at3(i, j, k, g);   // phi, phi_prev: natural; b, w: split
        const double x = phi[p];
        const double L = (nsum6n(phi, i, j, k, g) - 6.0 * x) * ih2;
        a[0] += (x * x) * (x * x);
        a[1] += x * x;
        a[2] += (phi[qe] - x) * (phi[qe] - x) + (phi[qn] - x) * (phi[qn] - x) +
                (phi[qt] - x) * (phi[qt] - x);
        a[3] += L * L;
        a[4] += x;
        if (phiprev) {
            const double d = x - phiprev[p];
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
