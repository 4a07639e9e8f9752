// libmpfc.so: host side of the MPFC nonlinear FAS multigrid time step on one
// gfx950 GPU, behind the C ABI declared in include/mpfc.h.
//
// A step of either convex-splitting scheme (Sec. 3.1, 3.2) solves N(u) = S
// (App. B.1, B.2) by FAS V(nu1, nu2) cycles: red-black nonlinear Gauss-Seidel
// smoothing, residual and 2x2-average restriction, FAS coarse right-hand
// side, direct solve on the coarsest grid, bilinear prolongation of the
// coarse-grid correction.  Levels above 32x32 cells take two fused tile
// launches per cycle (tiles.hpp); all smaller levels take one persistent
// launch.  One V-cycle is captured once into a hipGraph and replayed.  The
// stopping test runs on the device (the finest up-launch records the
// residual norm and raises a stop flag that every later kernel checks), so
// the host only reads back a small status record per cycle.  Afterwards psi
// is updated (eqs. discrete_1_b / discrete_2_b) and the energies of Sec. 3
// are computed, the -1 norm with the same multigrid on the Poisson problem.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mpfc.h"
#include "step.hpp"
#include "poisson.hpp"
#include "wrapup.hpp"
#include "launch.hpp"
#include "tiles.hpp"

using namespace mpfc;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(MPFC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}
int round_even(int v) { return (v + 1) & ~1; }

// Cells of the largest level the persistent coarse kernel takes.
int persistent_cells(const mpfc_opts* o) {
    return o->coarse_threshold ? o->coarse_threshold : CP_CELLS;
}

static_assert(BC_NEUMANN_X == MPFC_BC_NEUMANN_X && BC_NEUMANN_Y == MPFC_BC_NEUMANN_Y,
              "boundary-condition bits of the kernels and the C interface agree");
Grid make_grid(int m, int n, int bc) {
    return Grid{m, n, is_pow2(m) ? ilog2(m) : -1, is_pow2(n) ? ilog2(n) : -1, bc};
}
bool general_grid(const Grid& g) { return g.lm < 0 || g.ln < 0; }

// Levels of the hierarchy: coarsen while the smaller side exceeds `coarsest`
// and both sides of the next level stay even (a periodic red-black colouring
// needs an even number of cells per axis).  Powers of two end at the 2 x 2
// (or 2 x 4) grid; 512 x 400 ends at 64 x 50.
bool coarsen_more(int mm, int nn, int coarsest) {
    return (mm < nn ? mm : nn) > coarsest && mm % 4 == 0 && nn % 4 == 0;
}

constexpr int NT = 256;
const dim3 B2(64, 4);
dim3 grid2(int nx, int ny) { return dim3((nx + 63) / 64, (ny + 3) / 4); }
dim3 grid1(size_t total) { return dim3((unsigned)((total + 255) / 256)); }
// Workgroups of the grid-stride reductions (norms, energies): each writes its
// partial sums (up to 8 values) to `part`; one workgroup per CU left these
// passes latency bound.
constexpr unsigned kRedBlocks = 1024;
// Values per reduction workgroup in the step's wrap-up (k_wrap_rhs_terms).
constexpr unsigned kWrapSums = 12;
unsigned red_blocks(size_t total) {
    size_t b = (total + NT - 1) / NT;
    return (unsigned)(b < kRedBlocks ? b : kRedBlocks);
}

// Launch kinds that carry a tuned shape per level.
enum { SH_DN = 0, SH_UP = 1, SH_DN32 = 2, SH_UP32 = 3, SH_PDN = 4, SH_PUP = 5, SH_KINDS = 6 };

struct Level {
    int m = 0, n = 0;
    double h = 0;
    Grid g{};
    bool tiled = false;     // more than CP_CELLS cells: fused tile launches
    int shape[SH_KINDS] = {-1, -1, -1, -1, -1, -1};  // tile shape per launch kind (tuned)
    // MPFC system
    double* u[2][3] = {};   // ping-pong; u[0] holds the iterate between cycles
    double* v[3] = {};      // restricted iterate (coarse levels)
    double* f[3] = {};      // complete right-hand side (finest: S)
    double* rr[3] = {};     // restricted residual (coarse levels)
    double* xk = nullptr;   // phi^k on this level (scheme 2)
    double* pin = nullptr;  // pinning weight on this level (2x2 averages of the finest)
    // Poisson problem of the -1 norm
    double* w[2] = {};
    double* pv = nullptr;
    double* pf = nullptr;   // finest: b = psi - mean(psi)
    double* prr = nullptr;
};

struct CnnNet;               // learned-guess network (defined with its kernels)
void cnn_free(CnnNet* net);

}  // namespace

struct mpfc_ctx {
    int m = 0, n = 0;
    bool gen = false;           // a side is not a power of two (general-index kernels)
    mpfc_params p{};
    mpfc_opts o{};
    hipStream_t stream = nullptr;
    double c = 0, d = 0, alpha = 0;
    std::vector<Level> L;
    int Lp = 0;                 // first level handled by the persistent kernel
    double* phik = nullptr;     // copy of phi^k (finest)
    CycleState* st = nullptr;   // nonlinear cycle state
    double* hist = nullptr;     // device residual history
    CycleState* pst = nullptr;  // Poisson cycle state
    double* phist = nullptr;
    double* acc = nullptr;      // reduction results
    double* part = nullptr;     // per-block partial sums of the reductions
    bool pinned = false;        // pinning term of Sec. 4.6 active
    double* pin_mem = nullptr;  // weights of every level, then phi_hat (own allocation)
    double* phihat = nullptr;
    int nparts = 0;
    double* G = nullptr;        // coarsest Poisson Green's matrix
    int have_w = 0;
    int poisson_cycles = 3;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    double* host_buf = nullptr;     // pinned mirror of the readback block
    // Readback block: the cycle state (rb[0..7]), the Poisson state
    // (rb[8..15]), the reduction results `acc` (rb[16..31]) and the residual
    // history (rb[32..]), so that one copy returns all of them.
    double* rb = nullptr;
    size_t rb_count = 0;            // doubles of one full readback
    StepIO* io = nullptr;           // the caller's arrays of the current step
    // captured graphs (set-up, runs of cycles, Poisson cycle, wrap-up)
    bool use_graph = true;
    std::vector<std::pair<int, hipGraphExec_t>> graphs;
    hipStream_t cap_stream = nullptr;  // capture only (the caller's stream may be the null stream)
    // live timing of the finest-level launches (HIP events on `stream`)
    int prof = 0;
    hipEvent_t ev[4] = {};
    double prof_ms[2] = {0, 0};       // finest down, finest up
    long long prof_launches[2] = {0, 0};
    // mixed precision: FP32 correction cycles inside FP64 defect correction
    struct FLevel {
        float* e[2][3] = {};  // correction, ping-pong
        float* v[3] = {};
        float* f[3] = {};     // finest: FP64 residual rounded to FP32
        float* rr[3] = {};
        float* xk = nullptr;  // phi^k (FP32) on this level
        float* pb = nullptr;  // base phi (FP32) on this level
    };
    std::vector<FLevel> FL;
    int inner_cycles = 3;                  // FP32 cycles of the step's first outer iteration
    int inner_next = 3;                    // ... and of each later one
    int pred_units = 4;                    // cycles (outer iterations) the last step needed
    // learned initial guess (guess mode MPFC_GUESS_CNN)
    CnnNet* cnn = nullptr;
    double* cnn_r2 = nullptr;              // squared residual norms: [0] learned, [1] extrapolated
    unsigned long long* cnn_counts = nullptr;  // [0] steps that used the learned guess, [1] fallbacks
};

namespace {

// ---- operators per level --------------------------------------------------------
LevelOp<double> level_op(const mpfc_ctx* C, const Level& lv) {
    LevelOp<double> op;
    op.ih2 = 1.0 / (lv.h * lv.h);
    op.c = C->c;
    op.al = C->p.scheme == 1 ? C->alpha : 0.5 * C->alpha;
    op.e = C->p.scheme == 1 ? 1.0 : 0.5;
    op.w = C->o.omega;
    return op;
}

template <class Op>
Op make_op(const mpfc_ctx* C, const Level& lv) {
    if constexpr (Op::NF == 3) {
        Op o;
        o.op = level_op(C, lv);
        return o;
    } else {
        Op o;
        o.ih2 = 1.0 / (lv.h * lv.h);
        o.h2 = lv.h * lv.h;
        return o;
    }
}

Fields<double> finest_fields(const mpfc_ctx* C) {
    const Level& lv = C->L[0];
    Fields<double> F;
    F.phi = lv.u[0][0]; F.mu = lv.u[0][1]; F.ka = lv.u[0][2];
    F.f1 = lv.f[0]; F.f2 = lv.f[1]; F.f3 = lv.f[2];
    F.phik = C->p.scheme == 2 ? C->phik : nullptr;
    F.base = nullptr;
    F.pin = C->pinned ? lv.pin : nullptr;
    return F;
}

// First shape whose halo allowance covers H (used until the autotuner has run).
int pick_shape(int H) {
    for (int k = 0; k < kNumShapes; ++k)
        if (H <= kShapes[k].hmax) return k;
    return kNumShapes - 1;
}

// Tuned choice from the measured times: the first shape (in table order)
// within 5 % of the fastest, so that near-ties do not flip between runs.  The
// window is taken on |best|, so the fastest shape always qualifies, also when
// a time with the preceding launch's time subtracted comes out at or below 0.
int pick_tuned(const float* t, float best, int H) {
    for (int k = 0; k < kNumShapes; ++k)
        if (H <= kShapes[k].hmax && t[k] < 1e30f && t[k] <= best + 0.05f * std::fabs(best))
            return k;
    return pick_shape(H);
}

int level_shape(const Level& lv, int kind, int H) {
    const int k = lv.shape[kind];
    return (k >= 0 && H <= kShapes[k].hmax) ? k : pick_shape(H);
}

// Largest even divisor of `side` that is at most `cap` (side even).
int even_divisor(int side, int cap) {
    for (int d = cap < side ? cap : side; d >= 2; --d)
        if (d % 2 == 0 && side % d == 0) return d;
    return 2;
}

// Tile interior of a launch: the shape's sides, clamped to the level; on a
// general grid the largest even divisors of the level's sides within them.
void tile_dims(const Level& lv, int shape, int& tx, int& ty) {
    if (general_grid(lv.g)) {
        tx = even_divisor(lv.m, kShapes[shape].tx);
        ty = even_divisor(lv.n, kShapes[shape].ty);
        return;
    }
    tx = lv.m < kShapes[shape].tx ? lv.m : kShapes[shape].tx;
    ty = lv.n < kShapes[shape].ty ? lv.n : kShapes[shape].ty;
}

CoarseGeom coarse_geom(const mpfc_ctx* C) {
    CoarseGeom G{};
    G.bc = C->p.bc;
    G.nlev = (int)C->L.size() - C->Lp;
    int off = 0;
    for (int k = 0; k < G.nlev; ++k) {
        const Level& lv = C->L[C->Lp + k];
        G.m[k] = lv.m; G.n[k] = lv.n; G.lm[k] = lv.g.lm;
        G.off[k] = off;
        off += lv.m * lv.n;
    }
    return G;
}

void prof_mark(mpfc_ctx* C, int which, hipStream_t s) {
    (void)hipEventRecord(C->ev[which], s);
}

void prof_collect(mpfc_ctx* C) {
    for (int k = 0; k < 2; ++k) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, C->ev[2 * k], C->ev[2 * k + 1]) == hipSuccess) {
            C->prof_ms[k] += ms;
            C->prof_launches[k] += 1;
        }
    }
}

// ---- launch arguments of one level (shared by the single and batched paths) ------
// FP64 MPFC system, down launch of tiled level l: smooth, residual, restrict.
TileArgs<double> dn_args64(const mpfc_ctx* C, int l) {
    const Level& A = C->L[l];
    const Level& B = C->L[l + 1];
    TileArgs<double> T{};
    T.g = A.g;
    for (int f = 0; f < 3; ++f) {
        T.uin[f] = A.u[0][f];
        T.uout[f] = A.u[1][f];
        T.f[f] = l == 0 ? A.f[f] : A.rr[f];
        T.fout[f] = A.f[f];
        T.uH[f] = B.u[0][f];
        T.vH[f] = B.v[f];
        T.rH[f] = B.rr[f];
    }
    T.xk = A.xk;
    T.xkH = B.xk;  // phi^k of the next level (scheme 2), averaged in-kernel
    T.pin = C->pinned ? A.pin : nullptr;
    T.complete_f = l > 0;
    T.nsweep = 2 * C->o.nu1;
    T.H = round_even(T.nsweep + 1);
    return T;
}

// ... up launch: coarse-grid correction, smooth; the finest one also the norm.
TileArgs<double> up_args64(const mpfc_ctx* C, int l, bool norm) {
    const Level& A = C->L[l];
    const Level& B = C->L[l + 1];
    TileArgs<double> T{};
    T.g = A.g;
    for (int f = 0; f < 3; ++f) {
        T.uin[f] = A.u[1][f];
        T.uout[f] = A.u[0][f];
        T.f[f] = A.f[f];
        T.cuH[f] = B.u[0][f];
        T.cvH[f] = B.v[f];
    }
    T.xk = A.xk;
    T.pin = C->pinned ? A.pin : nullptr;
    T.nsweep = 2 * C->o.nu2;
    T.norm = norm;
    T.H = l == 0 ? round_even(T.nsweep + 1) : T.nsweep;
    T.part = C->part;
    return T;
}

// ... persistent launch: every level from Lp down.
CoarseArgs<double> coarse_args64(const mpfc_ctx* C) {
    const Level& top = C->L[C->Lp];
    CoarseArgs<double> A{};
    A.geo = coarse_geom(C);
    for (int f = 0; f < 3; ++f) {
        A.u[f] = top.u[0][f];
        A.rr[f] = C->Lp > 0 ? top.rr[f] : top.f[f];
    }
    A.xk = top.xk;
    A.pin = C->pinned ? top.pin : nullptr;
    A.h_top = top.h;
    A.nsw1 = 2 * C->o.nu1;
    A.nsw2 = 2 * C->o.nu2;
    A.complete_top = C->Lp > 0;
    A.newton_maxit = 30;
    A.newton_tol = 1e-15;
    return A;
}

// FP32 correction equation of mixed precision (same roles, FL buffers).
template <class Op>
Op make_op32(const mpfc_ctx* C, const Level& lv) {
    Op o;
    o.op.ih2 = (float)(1.0 / (lv.h * lv.h));
    o.op.c = (float)C->c;
    o.op.al = (float)(C->p.scheme == 1 ? C->alpha : 0.5 * C->alpha);
    o.op.e = (float)(C->p.scheme == 1 ? 1.0 : 0.5);
    o.op.w = (float)C->o.omega;
    return o;
}

TileArgs<float> dn_args32(const mpfc_ctx* C, int l) {
    const Level& A = C->L[l];
    const auto& FA = C->FL[l];
    const auto& FB = C->FL[l + 1];
    TileArgs<float> T{};
    T.g = A.g;
    for (int f = 0; f < 3; ++f) {
        T.uin[f] = FA.e[0][f];
        T.uout[f] = FA.e[1][f];
        T.f[f] = l == 0 ? FA.f[f] : FA.rr[f];
        T.fout[f] = FA.f[f];
        T.uH[f] = FB.e[0][f];
        T.vH[f] = FB.v[f];
        T.rH[f] = FB.rr[f];
    }
    T.xk = FA.xk;
    T.pb = FA.pb;
    T.xkH = FB.xk;  // coefficient fields of the next level, averaged in-kernel
    T.pbH = FB.pb;
    T.complete_f = l > 0;
    T.nsweep = 2 * C->o.nu1;
    T.H = round_even(T.nsweep + 1);
    // fewer passes below the finest level (the halo stays that of nu1, which
    // covers them: inner_nu_coarse <= nu1)
    if (l > 0 && C->o.inner_nu_coarse) T.nsweep = 2 * C->o.inner_nu_coarse;
    return T;
}

TileArgs<float> up_args32(const mpfc_ctx* C, int l) {
    const Level& A = C->L[l];
    const auto& FA = C->FL[l];
    const auto& FB = C->FL[l + 1];
    TileArgs<float> T{};
    T.g = A.g;
    for (int f = 0; f < 3; ++f) {
        T.uin[f] = FA.e[1][f];
        T.uout[f] = FA.e[0][f];
        T.f[f] = FA.f[f];
        T.cuH[f] = FB.e[0][f];
        T.cvH[f] = FB.v[f];
    }
    T.xk = FA.xk;
    T.pb = FA.pb;
    T.nsweep = 2 * C->o.nu2;
    T.norm = 0;
    T.H = T.nsweep;
    if (l > 0 && C->o.inner_nu_coarse) T.nsweep = 2 * C->o.inner_nu_coarse;  // H covers it
    return T;
}

CoarseArgs<float> coarse_args32(const mpfc_ctx* C) {
    const Level& top = C->L[C->Lp];
    const auto& FT = C->FL[C->Lp];
    CoarseArgs<float> A{};
    A.geo = coarse_geom(C);
    for (int f = 0; f < 3; ++f) {
        A.u[f] = FT.e[0][f];
        A.rr[f] = C->Lp > 0 ? FT.rr[f] : FT.f[f];
    }
    A.xk = FT.xk;
    A.pb = FT.pb;
    A.h_top = (float)top.h;
    A.nsw1 = 2 * C->o.nu1;
    A.nsw2 = 2 * C->o.nu2;
    if (C->Lp > 0 && C->o.inner_nu_coarse)  // every level here is below the finest
        A.nsw1 = A.nsw2 = 2 * C->o.inner_nu_coarse;
    A.complete_top = C->Lp > 0;
    A.newton_maxit = 20;
    A.newton_tol = 1e-6f;
    return A;
}

// Coarsest-grid cell count (4 or 8) selects the persistent kernel's direct solve.
bool coarsest_is_4(const mpfc_ctx* C) {
    const Level& cl = C->L.back();
    return cl.m * cl.n == 4;
}

// One FAS V-cycle of the MPFC system on all levels.  With `only` >= 0 just
// the down (only_up = 0) or up (1) launch of that level is issued, without
// the stop flag or the norm (used by the tile autotuner).
template <class Op>
void vcycle_mpfc_t(mpfc_ctx* C, hipStream_t s, int only = -1, int only_up = 0) {
    const int nl = (int)C->L.size(), Lp = C->Lp;
    const CycleState* stop = only >= 0 ? nullptr : C->st;
    for (int l = 0; l < Lp; ++l) {
        if (only >= 0 && (l != only || only_up)) continue;
        const Level& A = C->L[l];
        TileArgs<double> T = dn_args64(C, l);
        const int shape = level_shape(A, SH_DN, T.H);
        tile_dims(A, shape, T.tx, T.ty);
        if (l == 0 && C->prof) prof_mark(C, 0, s);
        launch_tile<Op, false>(make_op<Op>(C, A), T, shape, stop, s);
        if (l == 0 && C->prof) prof_mark(C, 1, s);
    }
    if (Lp < nl && only < 0) {
        CoarseArgs<double> A = coarse_args64(C);
        const Op op = make_op<Op>(C, C->L[Lp]);
        if (C->gen) {
            A.nsw2 = 2 * C->o.coarse_sweeps;
            launch_coarsest_gen<Op>(op, A, stop, s);
        } else {
            launch_coarse<Op>(op, A, coarsest_is_4(C), stop, s);
        }
    }
    for (int l = Lp - 1; l >= 0; --l) {
        if (only >= 0 && (l != only || !only_up)) continue;
        const Level& A = C->L[l];
        TileArgs<double> T = up_args64(C, l, l == 0 && only < 0);
        const int shape = level_shape(A, SH_UP, T.H);
        tile_dims(A, shape, T.tx, T.ty);
        if (l == 0 && C->prof) prof_mark(C, 2, s);
        launch_tile<Op, true>(make_op<Op>(C, A), T, shape, stop, s);
        if (l == 0 && C->prof) prof_mark(C, 3, s);
        if (T.norm) {
            const int nb = (A.m / T.tx) * (A.n / T.ty);
            hipLaunchKernelGGL((k_norm_finalize<NT>), dim3(1), dim3(NT), 0, s, C->part, nb, C->st,
                               C->hist, A.h * A.h, C->o.tol, C->o.max_cycles + 1, C->o.diverge);
        }
    }
}

void resnorm(mpfc_ctx* C, hipStream_t s) {
    const Level& lv = C->L[0];
    const size_t total = (size_t)lv.m * lv.n;
    const double h2 = lv.h * lv.h;
    const int max_norms = C->o.max_cycles + 1;
    const unsigned nb = red_blocks(total);
    if (C->p.scheme == 1)
        hipLaunchKernelGGL((k_resnorm<1, NT>), dim3(nb), dim3(NT), 0, s, finest_fields(C),
                           level_op(C, lv), lv.g, C->st, C->part, nullptr, nullptr, nullptr);
    else
        hipLaunchKernelGGL((k_resnorm<2, NT>), dim3(nb), dim3(NT), 0, s, finest_fields(C),
                           level_op(C, lv), lv.g, C->st, C->part, nullptr, nullptr, nullptr);
    hipLaunchKernelGGL((k_norm_finalize<NT>), dim3(1), dim3(NT), 0, s, C->part, (int)nb, C->st,
                       C->hist, h2, C->o.tol, max_norms, C->o.diverge);
}

// ---- mixed precision ---------------------------------------------------------------
// One FP32 FAS V-cycle on the correction equation N(u + e) - N(u) = r (DEFECT
// operators: the base phi of every level is a coefficient field).
template <class Op>
void vcycle_inner_t(mpfc_ctx* C, hipStream_t s, int only = -1, int only_up = 0,
                    bool first = false) {
    const int nl = (int)C->L.size(), Lp = C->Lp;
    const CycleState* stop = only >= 0 ? nullptr : C->st;
    for (int l = 0; l < Lp; ++l) {
        if (only >= 0 && (l != only || only_up)) continue;
        const Level& A = C->L[l];
        TileArgs<float> Tg = dn_args32(C, l);
        Tg.zero_in = first && l == 0;  // the outer iteration's correction starts at zero
        const int shape = level_shape(A, SH_DN32, Tg.H);
        tile_dims(A, shape, Tg.tx, Tg.ty);
        launch_tile<Op, false>(make_op32<Op>(C, A), Tg, shape, stop, s);
    }
    if (Lp < nl && only < 0) {
        const CoarseArgs<float> A = coarse_args32(C);
        const Op op = make_op32<Op>(C, C->L[Lp]);
        launch_coarse<Op>(op, A, coarsest_is_4(C), stop, s);
    }
    for (int l = Lp - 1; l >= 0; --l) {
        if (only >= 0 && (l != only || !only_up)) continue;
        const Level& A = C->L[l];
        TileArgs<float> Tg = up_args32(C, l);
        const int shape = level_shape(A, SH_UP32, Tg.H);
        tile_dims(A, shape, Tg.tx, Tg.ty);
        launch_tile<Op, true>(make_op32<Op>(C, A), Tg, shape, stop, s);
    }
}

// FP64 defect step on the finest grid: u[to] = u[from] + e (add) or u[from],
// r = S - N(u[to]) with its norm (stopping test), r and base phi to FP32.
void defect(mpfc_ctx* C, int from, int add, hipStream_t s) {
    const Level& F0 = C->L[0];
    const auto& FF = C->FL[0];
    const size_t total = (size_t)F0.m * F0.n;
    Fields<double> F;
    F.phi = F0.u[from][0]; F.mu = F0.u[from][1]; F.ka = F0.u[from][2];
    F.f1 = F0.f[0]; F.f2 = F0.f[1]; F.f3 = F0.f[2];
    F.phik = C->p.scheme == 2 ? C->phik : nullptr;
    F.base = nullptr;
    const int to = from ^ 1;
    const int max_norms = C->o.max_cycles + 1;
    // one 32 x 8 tile per workgroup (the partial sums hold one value per 256
    // cells), its values and their ring staged in LDS
    auto kern = C->p.scheme == 1 ? k_defect_tile<1> : k_defect_tile<2>;
    const dim3 grid((F0.m + DT_X - 1) / DT_X, (F0.n + DT_Y - 1) / DT_Y);
    const unsigned nb = grid.x * grid.y;
    hipLaunchKernelGGL(kern, grid, dim3(DT_X * DT_Y), 0, s, F, level_op(C, F0), F0.g, C->st,
                       C->part, FF.e[0][0], FF.e[0][1], FF.e[0][2], add, F0.u[to][0], F0.u[to][1],
                       F0.u[to][2], FF.f[0], FF.f[1], FF.f[2], FF.pb);
    hipLaunchKernelGGL((k_norm_finalize<NT>), dim3(1), dim3(NT), 0, s, C->part, (int)nb, C->st,
                       C->hist, F0.h * F0.h, C->o.tol, max_norms, C->o.diverge);
}

// One outer iteration of mixed precision starting from FP64 copy `from`:
// `ncyc` FP32 V-cycles on the correction (from e = 0), then the FP64 defect
// step into the other copy.
void outer_mixed(mpfc_ctx* C, int from, int ncyc, hipStream_t s) {
    const auto& FF = C->FL[0];
    const size_t total = (size_t)C->m * C->n;
    // The first inner cycle's finest down launch starts from e = 0 and its down
    // launches average the base phi onto the coarser levels; without tiled
    // levels the persistent kernel reads e from memory, so clear it.
    if (C->Lp == 0)
        for (int f = 0; f < 3; ++f)
            hipLaunchKernelGGL((k_fill<float>), grid1(total), dim3(256), 0, s, FF.e[0][f], total, 0.f);
    const bool nw = C->o.linearization == MPFC_NEWTON;
    for (int k = 0; k < ncyc; ++k) {
        const bool first = k == 0;
        if (C->p.scheme == 1) {
            if (nw) vcycle_inner_t<MpfcOp<float, 1, true, true>>(C, s, -1, 0, first);
            else vcycle_inner_t<MpfcOp<float, 1, false, true>>(C, s, -1, 0, first);
        } else {
            if (nw) vcycle_inner_t<MpfcOp<float, 2, true, true>>(C, s, -1, 0, first);
            else vcycle_inner_t<MpfcOp<float, 2, false, true>>(C, s, -1, 0, first);
        }
    }
    defect(C, from, 1, s);
}

void vcycle_mpfc(mpfc_ctx* C, hipStream_t s) {
    const bool nw = C->o.linearization == MPFC_NEWTON;
    if (C->p.scheme == 1) {
        if (nw) vcycle_mpfc_t<MpfcOp<double, 1, true, false>>(C, s);
        else vcycle_mpfc_t<MpfcOp<double, 1, false, false>>(C, s);
    } else if (C->pinned) {  // Sec. 4.6 pinning: scheme 2, Newton (checked when set)
        vcycle_mpfc_t<MpfcOp<double, 2, true, false, true>>(C, s);
    } else {
        if (nw) vcycle_mpfc_t<MpfcOp<double, 2, true, false>>(C, s);
        else vcycle_mpfc_t<MpfcOp<double, 2, false, false>>(C, s);
    }
    if (C->Lp == 0) resnorm(C, s);
}

// Stopping test of the Poisson solve of the -1 norm: ||r|| <= 1e-11 ||b||, or
// stalled at the rounding floor below 1e-8 ||b||; at most 60 cycles per step.
constexpr double kPoissonRel = 1e-11, kPoissonStall = 1e-8;
constexpr int kPoissonMax = 60;

// One V-cycle of the Poisson problem -Lap_h w = b (same structure, scalar).
void vcycle_poisson(mpfc_ctx* C, hipStream_t s, int only = -1, int only_up = 0) {
    using Op = PoissonOp<double>;
    const int nl = (int)C->L.size(), Lp = C->Lp;
    const CycleState* stop = only >= 0 ? nullptr : C->pst;
    for (int l = 0; l < Lp; ++l) {
        if (only >= 0 && (l != only || only_up)) continue;
        const Level& A = C->L[l];
        const Level& B = C->L[l + 1];
        TileArgs<double> T{};
        T.g = A.g;
        T.uin[0] = A.w[0]; T.uout[0] = A.w[1];
        T.f[0] = l == 0 ? A.pf : A.prr;
        T.fout[0] = A.pf;
        T.uH[0] = B.w[0]; T.vH[0] = B.pv; T.rH[0] = B.prr;
        T.complete_f = l > 0;
        T.nsweep = 4;
        T.H = 6;
        const int shape = level_shape(A, SH_PDN, T.H);
        tile_dims(A, shape, T.tx, T.ty);
        launch_tile<Op, false>(make_op<Op>(C, A), T, shape, stop, s);
    }
    if (Lp < nl && only < 0) {
        const Level& top = C->L[Lp];
        CoarseArgs<double> A{};
        A.geo = coarse_geom(C);
        A.u[0] = top.w[0];
        A.rr[0] = Lp > 0 ? top.prr : top.pf;
        A.h_top = top.h;
        A.nsw1 = 4;
        A.nsw2 = 4;
        A.complete_top = Lp > 0;
        A.G = C->G;
        if (C->gen)
            launch_coarsest_poisson(make_op<Op>(C, top), A, stop, s);
        else
            launch_coarse<Op>(make_op<Op>(C, top), A, true, stop, s);
    }
    for (int l = Lp - 1; l >= 0; --l) {
        if (only >= 0 && (l != only || !only_up)) continue;
        const Level& A = C->L[l];
        const Level& B = C->L[l + 1];
        TileArgs<double> T{};
        T.g = A.g;
        T.uin[0] = A.w[1]; T.uout[0] = A.w[0];
        T.f[0] = A.pf;
        T.cuH[0] = B.w[0]; T.cvH[0] = B.pv;
        T.nsweep = 4;
        T.norm = l == 0 && only < 0;
        T.H = l == 0 ? 6 : 4;
        T.part = C->part;
        const int shape = level_shape(A, SH_PUP, T.H);
        tile_dims(A, shape, T.tx, T.ty);
        launch_tile<Op, true>(make_op<Op>(C, A), T, shape, stop, s);
        if (T.norm) {
            const int nb = (A.m / T.tx) * (A.n / T.ty);
            hipLaunchKernelGGL((k_p_finalize<NT>), dim3(1), dim3(NT), 0, s, C->part, nb, C->pst,
                               C->phist, C->acc + 10, kPoissonRel, kPoissonStall, kPoissonMax);
        }
    }
    if (Lp == 0 && only < 0) {
        const Level& F0 = C->L[0];
        const unsigned nb = red_blocks((size_t)F0.m * F0.n);
        hipLaunchKernelGGL((k_p_resnorm<NT>), dim3(nb), dim3(NT), 0, s, F0.w[0], F0.pf, F0.g,
                           1.0 / (F0.h * F0.h), C->pst, C->part);
        hipLaunchKernelGGL((k_p_finalize<NT>), dim3(1), dim3(NT), 0, s, C->part, (int)nb, C->pst,
                           C->phist, C->acc + 10, kPoissonRel, kPoissonStall, kPoissonMax);
    }
}

// What one replayable unit of work is.
enum CycleKind { CYC_MPFC = 0, CYC_POISSON = 1 };

void enqueue(mpfc_ctx* C, int kind, hipStream_t s) {
    if (kind == CYC_MPFC) vcycle_mpfc(C, s);
    else vcycle_poisson(C, s);
}

// Unit `unit` (0, 1, ...) of a mixed-precision step: an outer iteration from
// FP64 copy 1 (even units; the set-up writes copy 1) or 0, with the first
// unit's FP32 cycle count or the later ones'.
void enqueue_outer(mpfc_ctx* C, int unit, hipStream_t s) {
    outer_mixed(C, 1 ^ (unit & 1), unit == 0 ? C->inner_cycles : C->inner_next, s);
}

// FP32 cycles that `nouter` outer iterations ran.
int inner_cycles_run(const mpfc_ctx* C, int nouter) {
    return nouter > 0 ? C->inner_cycles + (nouter - 1) * C->inner_next : 0;
}

// Captured graphs of a context, keyed by what they hold (graph_key): the
// step's set-up, runs of 1..kMaxRun V-cycles (or mixed-precision outer
// iterations, by the parity of the first one), one Poisson V-cycle, and the
// wrap-up variants.
enum GraphKind { GK_PROLOGUE = 1, GK_CYCLES = 2, GK_MIXED = 3, GK_POISSON = 4, GK_WRAPUP = 5 };
constexpr int kMaxRun = 8;
int graph_key(int kind, int a = 0, int b = 0) { return (kind * 16 + a) * 64 + b; }

void destroy_graphs(mpfc_ctx* C) {
    for (auto& g : C->graphs)
        if (g.second) (void)hipGraphExecDestroy(g.second);
    C->graphs.clear();
}

// Run the work `fn` enqueues: replayed from the graph captured under `key` on
// first use, or launched directly while profiling (or with graphs off).
template <class Fn>
int run_unit(mpfc_ctx* C, int key, Fn&& fn) {
    hipStream_t s = C->stream;
    if (!C->use_graph || C->prof) {
        fn(s);
        HIP_TRY(hipGetLastError());
        return MPFC_OK;
    }
    hipGraphExec_t gx = nullptr;
    for (auto& g : C->graphs)
        if (g.first == key) { gx = g.second; break; }
    if (!gx) {
        // Record the launches on a context-owned stream (nothing executes while
        // capturing), then replay the graph on the caller's stream.
        if (!C->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&C->cap_stream, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(C->cap_stream, hipStreamCaptureModeThreadLocal));
        fn(C->cap_stream);
        hipError_t le = hipGetLastError();
        hipError_t ce = hipStreamEndCapture(C->cap_stream, &g);
        if (le != hipSuccess || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(MPFC_EHIP, std::string("graph capture: ") +
                                       hipGetErrorString(le != hipSuccess ? le : ce));
        }
        hipError_t ie = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess)
            return fail(MPFC_EHIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
        C->graphs.emplace_back(key, gx);
    }
    HIP_TRY(hipGraphLaunch(gx, s));
    return MPFC_OK;
}

// One V-cycle of the Poisson problem of the -1 norm.
int run_poisson_cycle(mpfc_ctx* C) {
    return run_unit(C, graph_key(GK_POISSON), [&](hipStream_t s) { enqueue(C, CYC_POISSON, s); });
}

// `count` units of the step's solve (V-cycles, or mixed-precision outer
// iterations, the first being the step's unit number `first`), in runs of at
// most kMaxRun replayed from one graph each.  A mixed run's graph depends on
// the parity of its first unit and on whether it holds unit 0.
int run_cycles(mpfc_ctx* C, int first, int count) {
    const bool mixed = C->o.precision == MPFC_MIXED;
    while (count > 0) {
        const int k = count < kMaxRun ? count : kMaxRun;
        const int f0 = first;
        const int key = mixed ? graph_key(GK_MIXED, (f0 & 1) + (f0 == 0 ? 2 : 0), k)
                              : graph_key(GK_CYCLES, 0, k);
        int rc = run_unit(C, key, [&](hipStream_t s) {
            for (int j = 0; j < k; ++j) {
                if (mixed) enqueue_outer(C, f0 + j, s);
                else enqueue(C, CYC_MPFC, s);
            }
        });
        if (rc) return rc;
        first += k;
        count -= k;
    }
    return MPFC_OK;
}

// ---- tile-shape autotuner ----------------------------------------------------------
// Mean duration of one launch when `reps` launches run back to back from a
// graph, as inside a captured V-cycle.  Launching them from the host instead
// would time the host's submission rate for the small levels, whose kernels
// take a few microseconds.
template <class Fn>
int time_in_graph(hipStream_t& cap, hipStream_t s, int reps, Fn&& launch, float& ms) {
    if (!cap) HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    for (int r = 0; r < reps; ++r) launch(cap);
    const hipError_t le = hipGetLastError();
    const hipError_t ce = hipStreamEndCapture(cap, &g);
    if (le != hipSuccess || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(MPFC_EHIP, std::string("tuning graph capture: ") +
                                   hipGetErrorString(le != hipSuccess ? le : ce));
    }
    hipGraphExec_t gx = nullptr;
    const hipError_t ie = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return fail(MPFC_EHIP, std::string("tuning graph: ") + hipGetErrorString(ie));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipGraphLaunch(gx, s);  // warm
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < 2 && e == hipSuccess; ++r) e = hipGraphLaunch(gx, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float el = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&el, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipGraphExecDestroy(gx);
    if (e != hipSuccess) return fail(MPFC_EHIP, std::string("tuning: ") + hipGetErrorString(e));
    ms = el / (2.f * reps);
    return MPFC_OK;
}

constexpr int kTuneReps = 8;

// For every level with tile launches and every launch kind, time each tile
// shape whose halo allowance fits and keep the fastest (first within 5 %).
// The iterates do not depend on the shape (each cell's update is the same
// arithmetic in every tiling), so tuning changes speed only.
// `pre` launches the kernel that writes the candidate's inputs in a V-cycle
// (or nothing): each candidate launch is timed right after it, as in the
// cycle, where the inputs were just written (by other compute units) rather
// than left in cache by the candidate's own previous launch; the time of
// `pre` alone is subtracted.  Back-to-back launches of one small level favour
// large tiles that are slower inside the cycle.
// MPFC_TILE_SHAPE=<k> forces shape k instead.
template <class Fn, class Pre>
int tune_one(mpfc_ctx* C, Level& lv, int kind, int H, Fn&& launch, Pre&& pre, bool has_pre) {
    float t[kNumShapes];
    for (int k = 0; k < kNumShapes; ++k) t[k] = 1e30f;
    float t_pre = has_pre ? 1e30f : 0.f;
    // two interleaved rounds; each shape's faster one counts, and so does the
    // faster of the two timings of `pre` (the launches of the small levels
    // take a few microseconds, and a stall of the host between the timed
    // graph launches only ever adds time)
    for (int round = 0; round < 2; ++round) {
        if (has_pre) {
            float ms = 0.f;
            int rc = time_in_graph(C->cap_stream, C->stream, kTuneReps, pre, ms);
            if (rc) return rc;
            t_pre = ms < t_pre ? ms : t_pre;
        }
        for (int k = 0; k < kNumShapes; ++k) {
            if (H > kShapes[k].hmax || (C->gen && !gen_shape(k))) continue;
            lv.shape[kind] = k;
            float ms = 0.f;
            int rc = has_pre ? time_in_graph(C->cap_stream, C->stream, kTuneReps,
                                             [&](hipStream_t s) { pre(s); launch(s); }, ms)
                             : time_in_graph(C->cap_stream, C->stream, kTuneReps, launch, ms);
            if (rc) return rc;
            t[k] = ms < t[k] ? ms : t[k];
        }
    }
    float best = 1e30f;
    for (int k = 0; k < kNumShapes; ++k)
        if (t[k] < 1e30f) {
            t[k] -= t_pre;
            best = t[k] < best ? t[k] : best;
        }
    lv.shape[kind] = pick_tuned(t, best, H);
    return MPFC_OK;
}

int autotune(mpfc_ctx* C) {
    const char* forced = std::getenv("MPFC_TILE_SHAPE");
    if (forced && forced[0]) {
        const int k = std::atoi(forced);
        if (k < 0 || k >= kNumShapes) return fail(MPFC_EINVAL, "MPFC_TILE_SHAPE out of range");
        if (C->gen && !gen_shape(k))
            return fail(MPFC_EINVAL, "MPFC_TILE_SHAPE: grids with a side that is not a power of two "
                                     "take shape 0 or 2");
        for (auto& lv : C->L)
            for (int kind = 0; kind < SH_KINDS; ++kind) lv.shape[kind] = k;
        return MPFC_OK;
    }
    const bool nw = C->o.linearization == MPFC_NEWTON;
    const int Hd = round_even(2 * C->o.nu1 + 1), Hu = round_even(2 * C->o.nu2 + 1);
    // one launch of level `lev` (down or up) of the FP64 cycle, of the FP32
    // correction cycle and of the Poisson cycle
    auto f64 = [&](hipStream_t s, int lev, int up) {
        if (C->p.scheme == 1) {
            if (nw) vcycle_mpfc_t<MpfcOp<double, 1, true, false>>(C, s, lev, up);
            else vcycle_mpfc_t<MpfcOp<double, 1, false, false>>(C, s, lev, up);
        } else {
            if (nw) vcycle_mpfc_t<MpfcOp<double, 2, true, false>>(C, s, lev, up);
            else vcycle_mpfc_t<MpfcOp<double, 2, false, false>>(C, s, lev, up);
        }
    };
    auto f32 = [&](hipStream_t s, int lev, int up) {
        if (C->p.scheme == 1) {
            if (nw) vcycle_inner_t<MpfcOp<float, 1, true, true>>(C, s, lev, up);
            else vcycle_inner_t<MpfcOp<float, 1, false, true>>(C, s, lev, up);
        } else {
            if (nw) vcycle_inner_t<MpfcOp<float, 2, true, true>>(C, s, lev, up);
            else vcycle_inner_t<MpfcOp<float, 2, false, true>>(C, s, lev, up);
        }
    };
    // Levels in order, down before up: the kernel that writes a candidate's
    // inputs (the down launch of the level above for a down launch, the same
    // level's down launch for an up launch) is tuned before it.  The finest
    // down launch is timed alone.
    for (int l = 0; l < C->Lp; ++l) {
        Level& lv = C->L[l];
        for (int up = 0; up < 2; ++up) {
            const int H = up ? (l == 0 ? Hu : 2 * C->o.nu2) : Hd;
            const int pl = up ? l : l - 1;  // level of the preceding down launch
            const bool has_pre = pl >= 0;
            int rc = tune_one(
                C, lv, up ? SH_UP : SH_DN, H, [&](hipStream_t s) { f64(s, l, up); },
                [&](hipStream_t s) { f64(s, pl, 0); }, has_pre);
            if (rc) return rc;
            if (C->o.precision == MPFC_MIXED) {
                const int H32 = up ? 2 * C->o.nu2 : Hd;
                rc = tune_one(
                    C, lv, up ? SH_UP32 : SH_DN32, H32, [&](hipStream_t s) { f32(s, l, up); },
                    [&](hipStream_t s) { f32(s, pl, 0); }, has_pre);
                if (rc) return rc;
            }
            if (C->o.energy) {
                rc = tune_one(
                    C, lv, up ? SH_PUP : SH_PDN, up ? (l == 0 ? 6 : 4) : 6,
                    [&](hipStream_t s) { vcycle_poisson(C, s, l, up); },
                    [&](hipStream_t s) { vcycle_poisson(C, s, pl, 0); }, has_pre);
                if (rc) return rc;
            }
        }
    }
    HIP_TRY(hipGetLastError());
    return MPFC_OK;
}

// Mean-zero Green's matrix of -Lap_h on an m x n grid of spacing h with the
// boundary conditions `bc`, from the eigen-decomposition of the separable
// operator: G_pq = sum over modes k != 0 of v_k(p) v_k(q) / lambda_k.  Per
// axis of N cells, periodic: v_j(i) v_j(i') summed over the pair j, N - j is
// cos(2 pi j (i - i') / N) / N with lambda = (4/h^2) sin^2(pi j / N);
// Neumann: cosine modes w_j^2 cos(pi j (i + 1/2) / N) cos(pi j (i' + 1/2) / N),
// w_0^2 = 1/N, w_j^2 = 2/N, lambda = (4/h^2) sin^2(pi j / (2N)).
void green_matrix(int m, int n, double h, int bc, std::vector<double>& G) {
    const int N = m * n;
    G.assign((size_t)N * N, 0.0);
    const double pi = 3.14159265358979323846;
    auto mode = [&](int len, bool neumann, int j, int i, int i2, double& lam) {
        if (!neumann) {
            const double sn = std::sin(pi * j / len);
            lam = 4.0 / (h * h) * sn * sn;
            return std::cos(2.0 * pi * j * (double)(i - i2) / len) / len;
        }
        const double sn = std::sin(pi * j / (2.0 * len));
        lam = 4.0 / (h * h) * sn * sn;
        const double w2 = j == 0 ? 1.0 / len : 2.0 / len;
        return w2 * std::cos(pi * j * (i + 0.5) / len) * std::cos(pi * j * (i2 + 0.5) / len);
    };
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            double s = 0.0;
            for (int p = 0; p < m; ++p)
                for (int q = 0; q < n; ++q) {
                    if (p == 0 && q == 0) continue;
                    double lx, ly;
                    const double vx = mode(m, bc & BC_NEUMANN_X, p, a % m, b % m, lx);
                    const double vy = mode(n, bc & BC_NEUMANN_Y, q, a / m, b / m, ly);
                    s += vx * vy / (lx + ly);
                }
            G[(size_t)a * N + b] = s;
        }
}

// Separable eigenbasis of -Lap_h on an m x n grid (general grids' coarsest
// Poisson solve): G = [V_x (m x m) | V_y (n x n) | 1/lam (n x m)], V[i][k] =
// value of orthonormal mode k at cell i.  Periodic axis of N cells: mode 0 =
// 1/sqrt(N), modes 2j-1, 2j = sqrt(2/N) cos, sin(2 pi j i / N) (j < N/2),
// mode N-1 = (-1)^i / sqrt(N) (N even), each with lambda = (4/h^2)
// sin^2(pi j / N); Neumann: sqrt(w_k) cos(pi k (i + 1/2) / N), lambda =
// (4/h^2) sin^2(pi k / (2N)).  1/lam of the (0, 0) mode is 0.
void spectral_factors(int m, int n, double h, int bc, std::vector<double>& G) {
    const double pi = 3.14159265358979323846;
    G.assign((size_t)m * m + (size_t)n * n + (size_t)m * n, 0.0);
    auto basis = [&](int N, bool neumann, double* V, std::vector<double>& lam) {
        lam.assign(N, 0.0);
        for (int k = 0; k < N; ++k) {
            int j;             // frequency of mode k
            if (neumann) j = k;
            else j = k == 0 ? 0 : (k == N - 1 ? N / 2 : (k + 1) / 2);
            const double sn = neumann ? std::sin(pi * j / (2.0 * N)) : std::sin(pi * j / N);
            lam[k] = 4.0 / (h * h) * sn * sn;
            for (int i = 0; i < N; ++i) {
                double v;
                if (neumann) {
                    v = (k == 0 ? std::sqrt(1.0 / N) : std::sqrt(2.0 / N)) *
                        std::cos(pi * k * (i + 0.5) / N);
                } else if (k == 0) {
                    v = std::sqrt(1.0 / N);
                } else if (k == N - 1) {
                    v = ((i & 1) ? -1.0 : 1.0) / std::sqrt((double)N);
                } else {
                    const double a = 2.0 * pi * j * i / N;
                    v = std::sqrt(2.0 / N) * ((k & 1) ? std::cos(a) : std::sin(a));
                }
                V[(size_t)i * N + k] = v;
            }
        }
    };
    std::vector<double> lx, ly;
    basis(m, bc & BC_NEUMANN_X, G.data(), lx);
    basis(n, bc & BC_NEUMANN_Y, G.data() + (size_t)m * m, ly);
    double* il = G.data() + (size_t)m * m + (size_t)n * n;
    for (int l = 0; l < n; ++l)
        for (int k = 0; k < m; ++k)
            il[(size_t)l * m + k] = (l == 0 && k == 0) ? 0.0 : 1.0 / (lx[k] + ly[l]);
}

// Coefficients of the decoupled schemes (eqs. discrete_1_a, discrete_2_a):
// with q = 1 (first-order scheme) or 2 (second-order scheme),
// c = s M / (beta + q/s) on Lap mu, and d = q / (beta + q/s) on psi^k in S^(1).
void scheme_coefficients(const mpfc_params* p, double& c, double& d) {
    const double q = p->scheme == 1 ? 1.0 : 2.0;
    c = p->dt * p->M / (p->beta + q / p->dt);
    d = q / (p->beta + q / p->dt);
}

// Physical parameters alone (shared by the context and the operator-level
// entry points).
int validate_params(const mpfc_params* p) {
    if (!p) return fail(MPFC_EINVAL, "params is NULL");
    if (!(p->scheme == 1 || p->scheme == 2)) return fail(MPFC_EINVAL, "scheme must be 1 or 2");
    if (!(p->h > 0) || !std::isfinite(p->h)) return fail(MPFC_EINVAL, "h must be > 0");
    if (!(p->dt > 0) || !std::isfinite(p->dt)) return fail(MPFC_EINVAL, "dt must be > 0");
    if (!(p->M > 0) || !std::isfinite(p->M)) return fail(MPFC_EINVAL, "M must be > 0");
    if (!(p->beta >= 0) || !std::isfinite(p->beta)) return fail(MPFC_EINVAL, "beta must be >= 0");
    if (!(p->eps <= 1.0) || !std::isfinite(p->eps)) return fail(MPFC_EINVAL, "eps must be <= 1");
    if (p->bc < 0 || p->bc > (MPFC_BC_NEUMANN_X | MPFC_BC_NEUMANN_Y))
        return fail(MPFC_EINVAL, "bc must combine MPFC_BC_NEUMANN_X and MPFC_BC_NEUMANN_Y bits");
    return MPFC_OK;
}

// Operator constants of a grid of spacing p->h (LevelOp of the tile kernels).
LevelOp<double> params_op(const mpfc_params* p) {
    double c, d;
    scheme_coefficients(p, c, d);
    const double alpha = 1.0 - p->eps;
    LevelOp<double> op;
    op.ih2 = 1.0 / (p->h * p->h);
    op.c = c;
    op.al = p->scheme == 1 ? alpha : 0.5 * alpha;
    op.e = p->scheme == 1 ? 1.0 : 0.5;
    return op;
}

int validate(int m, int n, const mpfc_params* p, const mpfc_opts* o) {
    int prc = validate_params(p);
    if (prc) return prc;
    if (!o) return fail(MPFC_EINVAL, "opts is NULL");
    const bool gen = !(is_pow2(m) && is_pow2(n));
    if (m < 2 || n < 2) return fail(MPFC_EINVAL, "m and n must be >= 2");
    if (gen && (m % 4 != 0 || n % 4 != 0))
        return fail(MPFC_EINVAL, "m and n must be powers of two or multiples of 4");
    if ((long long)m * n > (1LL << 28)) return fail(MPFC_EINVAL, "grid too large (m*n > 2^28)");
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 < 1 || o->nu1 > 4 || o->nu2 > 4)
        return fail(MPFC_EINVAL, "nu1, nu2 must be in [0, 4] with nu1 + nu2 >= 1");
    if (o->max_cycles < 1 || o->max_cycles > 100000)
        return fail(MPFC_EINVAL, "max_cycles must be in [1, 100000]");
    if (!(o->tol > 0)) return fail(MPFC_EINVAL, "tol must be > 0");
    if (o->coarsest != 2) return fail(MPFC_EINVAL, "coarsest must be 2");
    if (!(o->precision == MPFC_FP64 || o->precision == MPFC_MIXED))
        return fail(MPFC_EINVAL, "precision must be MPFC_FP64 or MPFC_MIXED");
    if (!(o->guess == MPFC_GUESS_PREV || o->guess == MPFC_GUESS_EXTRAP ||
          o->guess == MPFC_GUESS_CNN))
        return fail(MPFC_EINVAL, "unknown guess mode");
    if (o->guess == MPFC_GUESS_CNN && p->bc != 0)
        return fail(MPFC_EINVAL, "the learned guess (periodic convolutions) needs periodic boundaries");
    if (!(o->linearization == MPFC_NEWTON || o->linearization == MPFC_PICARD))
        return fail(MPFC_EINVAL, "unknown linearization");
    if (!(o->diverge > 1.0)) return fail(MPFC_EINVAL, "diverge must be > 1");
    if (o->inner_cycles < 1 || o->inner_cycles > 16)
        return fail(MPFC_EINVAL, "inner_cycles must be in [1, 16]");
    if (o->inner_cycles_next < 0 || o->inner_cycles_next > 16)
        return fail(MPFC_EINVAL, "inner_cycles_next must be in [0, 16]");
    if (o->inner_nu_coarse < 0 || o->inner_nu_coarse > o->nu1 || o->inner_nu_coarse > o->nu2)
        return fail(MPFC_EINVAL, "inner_nu_coarse must be in [0, min(nu1, nu2)]");
    if (o->coarse_sweeps < 1 || o->coarse_sweeps > 64)
        return fail(MPFC_EINVAL, "coarse_sweeps must be in [1, 64]");
    if (!(o->omega > 0.0 && o->omega < 2.0))
        return fail(MPFC_EINVAL, "omega must be in (0, 2)");
    const int thr = o->coarse_threshold;
    if (thr != 0 && (gen || !is_pow2(thr) || thr < 256 || thr > CP_CELLS))
        return fail(MPFC_EINVAL, "coarse_threshold must be 0 or a power of two in [256, 1024] "
                                 "(power-of-two grids)");
    if (gen) {
        // general-index kernels: FP64, halos up to 6, coarsest level in one workgroup
        if (o->precision != MPFC_FP64)
            return fail(MPFC_EINVAL, "grids with a side that is not a power of two run in MPFC_FP64");
        if (o->guess == MPFC_GUESS_CNN)
            return fail(MPFC_EINVAL, "the learned guess needs power-of-two grids");
        if (o->nu1 > 2 || o->nu2 > 2)
            return fail(MPFC_EINVAL, "nu1, nu2 must be at most 2 when a side is not a power of two");
        int gm = m, gn = n;
        while (coarsen_more(gm, gn, o->coarsest)) { gm /= 2; gn /= 2; }
        if (gm * gn > CG_CELLS)
            return fail(MPFC_EINVAL, "the coarsest level (coarsened while both sides stay even) "
                                     "exceeds 4096 cells");
        return MPFC_OK;
    }
    // coarsest grid: coarsen while the smaller side exceeds `coarsest`
    int mm = m, nn = n;
    while ((mm < nn ? mm : nn) > o->coarsest) { mm /= 2; nn /= 2; }
    if (mm * nn > 8)
        return fail(MPFC_EINVAL, "aspect ratio above 2: the coarsest grid must be 2x2 or 2x4");
    // the levels of at most coarse_threshold cells must fit the persistent kernel
    const int cp = persistent_cells(o);
    int cells = 0;
    mm = m; nn = n;
    for (;;) {
        if (mm * nn <= cp) cells += mm * nn;
        if ((mm < nn ? mm : nn) <= o->coarsest) break;
        mm /= 2; nn /= 2;
    }
    if (cells > CP_TOTAL) return fail(MPFC_EINVAL, "internal: coarse levels exceed the LDS budget");
    return MPFC_OK;
}

int status_code(int st) {
    switch (st) {
        case ST_CONVERGED: return MPFC_OK;
        case ST_MAXCYC: return MPFC_ENOTCONVERGED;
        case ST_NONFINITE: return MPFC_ENONFINITE;
        case ST_DIVERGED: return MPFC_EDIVERGED;
        default: return MPFC_ENOTCONVERGED;
    }
}

// Energies from the reduction results a[0..7] (k_energy_terms) into out[0..3]:
// F (eq. discrete_energy_PFC, with pinning plus h^2 sum W (phi - phi_hat)^2),
// the pseudo energy F + ||psi||_{-1}^2 / (2M) (eq. discrete_energy_MPFC), the
// modified energy (eq. energy_numer) and the mass h^2 sum phi.
void energies_from_sums(const mpfc_ctx* C, const double* a, double* out) {
    const double h2 = C->L[0].h * C->L[0].h;
    const double Fe = 0.25 * h2 * a[0] + 0.5 * C->alpha * h2 * a[1] - a[2] + 0.5 * h2 * a[3] +
                      h2 * a[7];
    const double nm1 = h2 * a[6];
    out[0] = Fe;
    out[1] = Fe + nm1 / (2.0 * C->p.M);
    out[2] = out[1] + 0.5 * a[5];
    out[3] = h2 * a[4];
}

// Enqueue up front as many Poisson cycles as the last solve ran (0 when the
// warm start alone passed): skipped cycles still cost their launches, and
// each count is a graph of its own.
void adapt_poisson_cycles(mpfc_ctx* C, const CycleState& pst, bool warm) {
    const int ran = pst.count - (warm ? 1 : 0);  // V-cycles that ran
    C->poisson_cycles = ran < kMaxRun ? ran : kMaxRun;
}

// Energies of (phi, phi_prev, psi) into out[0..3] (mpfc_energies): the
// Poisson problem of the -1 norm is solved from the context's last solution
// (or from zero before the first).
int compute_energies(mpfc_ctx* C, const double* phi, const double* phiprev, const double* psi,
                     double* out) {
    hipStream_t s = C->stream;
    Level& F0 = C->L[0];
    const size_t total = (size_t)C->m * C->n;
    const unsigned rb = red_blocks(total);
    const bool warm = C->have_w != 0;
    // sum of psi (acc[8]), Poisson state reset; b = psi - mean and the sums of
    // b^2 and of the warm start's squared residual (acc[10], acc[11])
    hipLaunchKernelGGL((k_sum2<NT>), dim3(rb), dim3(NT), 0, s, psi, (const double*)nullptr, total,
                       C->part, C->pst);
    hipLaunchKernelGGL((k_partials_sum<NT>), dim3(1), dim3(NT), 0, s, C->part, (int)rb, 2, C->acc + 8);
    if (!warm)
        hipLaunchKernelGGL((k_fill<double>), grid1(total), dim3(256), 0, s, F0.w[0], total, 0.0);
    hipLaunchKernelGGL((k_p_rhs_resid<NT>), dim3(rb), dim3(NT), 0, s, F0.g, 1.0 / (F0.h * F0.h),
                       psi, C->acc + 8, F0.pf, warm ? F0.w[0] : nullptr, C->part);
    hipLaunchKernelGGL((k_partials_sum<NT>), dim3(1), dim3(NT), 0, s, C->part, (int)rb, 2,
                       C->acc + 10);
    // the warm start may already meet the stopping test (its residual is the
    // first norm of the solve)
    if (warm)
        hipLaunchKernelGGL((k_p_finalize<NT>), dim3(1), dim3(NT), 0, s, C->acc + 11, 1, C->pst,
                           C->phist, C->acc + 10, kPoissonRel, kPoissonStall, kPoissonMax);
    HIP_TRY(hipGetLastError());
    auto terms = [&]() -> int {
        hipLaunchKernelGGL((k_energy_terms<NT>), dim3(rb), dim3(NT), 0, s, F0.g,
                           1.0 / (F0.h * F0.h), phi, phiprev, F0.pf, F0.w[0], C->part,
                           (const double*)(C->pinned ? F0.pin : nullptr),
                           (const double*)(C->pinned ? C->phihat : nullptr));
        hipLaunchKernelGGL((k_partials_sum<NT>), dim3(1), dim3(NT), 0, s, C->part, (int)rb, 8,
                           C->acc);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(C->host_buf, C->rb, 32 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return MPFC_OK;
    };
    int launched = 0;
    for (int k = 0; k < C->poisson_cycles; ++k, ++launched) {
        int rc = run_poisson_cycle(C);
        if (rc) return rc;
    }
    int rc = terms();
    if (rc) return rc;
    const CycleState* hp = (const CycleState*)(C->host_buf + 8);
    while (!hp->done && launched < kPoissonMax) {
        for (int k = 0; k < 2; ++k, ++launched) {
            rc = run_poisson_cycle(C);
            if (rc) return rc;
        }
        rc = terms();
        if (rc) return rc;
    }
    const bool ok = hp->status == ST_CONVERGED;
    adapt_poisson_cycles(C, *hp, warm);
    C->have_w = 1;
    energies_from_sums(C, C->host_buf + 16, out);
    if (!ok) return fail(MPFC_ENOTCONVERGED, "Poisson solve of the -1 norm did not converge");
    return MPFC_OK;
}

int cnn_candidate(mpfc_ctx* C, const StepIO* io, hipStream_t s);
void cnn_choose(mpfc_ctx* C, hipStream_t s);

// ---- one step, split for reuse by the batched path -------------------------------
// Source (also copies phi^k), guess and its completion, stop state reset and
// the first residual norm (FP64), or for mixed precision phi^k in FP32 and the
// first FP64 defect (copy 0 -> 1).  The coarse levels' phi^k (scheme 2) is
// averaged by each cycle's down launches.  The caller's arrays are read from
// C->io (k_set_io), so the set-up is captured once and replayed.
int step_prologue(mpfc_ctx* C, hipStream_t s) {
    Level& F0 = C->L[0];
    const Grid g0 = F0.g;
    const size_t total = (size_t)C->m * C->n;
    const double ih2 = 1.0 / (F0.h * F0.h);
    const double e = C->p.scheme == 1 ? 1.0 : 0.5;
    const double al = C->p.scheme == 1 ? C->alpha : 0.5 * C->alpha;
    const bool learned = C->o.guess == MPFC_GUESS_CNN;
    const int gmode = C->o.guess == MPFC_GUESS_PREV ? 0 : 1;
    const double* pin = C->pinned ? F0.pin : nullptr;
    const double* phihat = C->pinned ? C->phihat : nullptr;
    // On sides that are multiples of 32 (x) and 8 (y): the whole set-up of the
    // extrapolated (or previous-step) guess in one tiled pass, with the first
    // norm's sums unless mixed precision forms its own first defect or the
    // learned guess is compared with it (then it goes to copy 1, and the
    // network's candidate to copy 0; both paths complete that guess with the
    // same arithmetic, so a network that falls back reproduces the run
    // without it bit for bit).
    if (F0.m % SU_X == 0 && F0.n % SU_Y == 0) {
        const dim3 grid(F0.m / SU_X, F0.n / SU_Y);
        const unsigned nb = grid.x * grid.y;
        const bool mixed = C->o.precision == MPFC_MIXED;
        const bool norm = !mixed && !learned;
        const int ce = learned ? 1 : 0;
        auto kern = C->p.scheme == 1 ? (norm ? k_setup_tile<1, true> : k_setup_tile<1, false>)
                                     : (norm ? k_setup_tile<2, true> : k_setup_tile<2, false>);
        hipLaunchKernelGGL(kern, grid, dim3(SU_X * SU_Y), 0, s, g0, level_op(C, F0), C->d,
                           C->alpha, gmode, (const StepIO*)C->io, F0.f[0], F0.f[1], F0.f[2],
                           C->phik, pin, phihat, F0.u[ce][0], F0.u[ce][2], F0.u[ce][1], C->st,
                           C->part);
        if (learned) {
            int rc = cnn_candidate(C, (const StepIO*)C->io, s);  // into copy 0, completed
            if (rc) return rc;
            cnn_choose(C, s);  // leaves the kept guess's sum in part[0]
        }
        if (!mixed) {
            hipLaunchKernelGGL((k_norm_finalize<NT>), dim3(1), dim3(NT), 0, s, C->part,
                               learned ? 1 : (int)nb, C->st, C->hist, F0.h * F0.h, C->o.tol,
                               C->o.max_cycles + 1, C->o.diverge);
        } else {
            const auto& FF = C->FL[0];
            if (C->p.scheme == 2)
                hipLaunchKernelGGL((k_convert<double, float>), grid1(total), dim3(256), 0, s,
                                   C->phik, FF.xk, total);
            defect(C, 0, 0, s);
        }
        HIP_TRY(hipGetLastError());
        return MPFC_OK;
    }
    // Source, guess and kappa in one pass (the caller's arrays from C->io: this
    // part is captured once and replayed); with the learned guess the
    // extrapolated candidate goes to copy 1 and the network's to copy 0.
    const int ce = learned ? 1 : 0;
    if (C->p.scheme == 1)
        hipLaunchKernelGGL((k_setup<1>), grid2(C->m, C->n), B2, 0, s, g0, ih2, C->d, C->alpha, e,
                           gmode, (const StepIO*)C->io, F0.f[0], F0.f[1], F0.f[2], C->phik,
                           (const double*)nullptr, (const double*)nullptr, F0.u[ce][0],
                           F0.u[ce][2], C->st);
    else
        hipLaunchKernelGGL((k_setup<2>), grid2(C->m, C->n), B2, 0, s, g0, ih2, C->d, C->alpha, e,
                           gmode, (const StepIO*)C->io, F0.f[0], F0.f[1], F0.f[2], C->phik, pin,
                           phihat, F0.u[ce][0], F0.u[ce][2], C->st);
    if (C->p.scheme == 1)
        hipLaunchKernelGGL((k_complete_mu<1>), grid2(C->m, C->n), B2, 0, s, g0, ih2, al,
                           F0.u[ce][0], C->phik, F0.u[ce][2], F0.f[1], F0.u[ce][1],
                           (const double*)nullptr);
    else
        hipLaunchKernelGGL((k_complete_mu<2>), grid2(C->m, C->n), B2, 0, s, g0, ih2, al,
                           F0.u[ce][0], C->phik, F0.u[ce][2], F0.f[1], F0.u[ce][1],
                           (const double*)(C->pinned ? F0.pin : nullptr));
    if (learned) {
        int rc = cnn_candidate(C, (const StepIO*)C->io, s);  // into copy 0, completed
        if (rc) return rc;
        cnn_choose(C, s);
    }
    if (C->o.precision != MPFC_MIXED) {
        if (learned) {  // the pick left the kept guess's squared norm in part[0]
            hipLaunchKernelGGL((k_norm_finalize<NT>), dim3(1), dim3(NT), 0, s, C->part, 1, C->st,
                               C->hist, F0.h * F0.h, C->o.tol, C->o.max_cycles + 1, C->o.diverge);
        } else {
            // the completed guess satisfies N^(2) = S^(2), N^(3) = S^(3): only r1 is left
            const unsigned nb = red_blocks(total);
            hipLaunchKernelGGL((k_resnorm_guess<NT>), dim3(nb), dim3(NT), 0, s, finest_fields(C),
                               level_op(C, F0), g0, C->part);
            hipLaunchKernelGGL((k_norm_finalize<NT>), dim3(1), dim3(NT), 0, s, C->part, (int)nb,
                               C->st, C->hist, F0.h * F0.h, C->o.tol, C->o.max_cycles + 1,
                               C->o.diverge);
        }
    } else {
        const auto& FF = C->FL[0];
        // the coarse levels' phi^k is averaged by the down launches of each cycle
        if (C->p.scheme == 2)
            hipLaunchKernelGGL((k_convert<double, float>), grid1(total), dim3(256), 0, s, C->phik,
                               FF.xk, total);
        defect(C, 0, 0, s);
    }
    HIP_TRY(hipGetLastError());
    return MPFC_OK;
}

void enqueue_energy_terms(mpfc_ctx* C, hipStream_t s, bool warm);

// Wrap-up of a step, enqueued behind its cycles (every kernel gated on the
// step's cycle state, wrapup.hpp): psi^{k+1} and phi^{k+1} into the caller's
// arrays, then (energies on) the -1 norm's Poisson problem, warm-started from
// the last step's solution by the scheme's relation between psi and mu
// (k_wrap_w_advance) or from zero (`warm` false), with `npoisson` V-cycles up
// front, and the energy sums.  The readback block then holds all results.
void enqueue_wrapup(mpfc_ctx* C, hipStream_t s, bool warm, int npoisson) {
    Level& F0 = C->L[0];
    const size_t total = (size_t)C->m * C->n;
    const int mixed = C->o.precision == MPFC_MIXED;
    const StepIO* io = C->io;
    WrapFields wf;
    for (int c = 0; c < 2; ++c) {
        wf.phi[c] = F0.u[c][0];
        wf.mu[c] = F0.u[c][1];
        wf.kappa[c] = F0.u[c][2];
    }
    if (!C->o.energy) {
        if (C->p.scheme == 1)
            hipLaunchKernelGGL((k_wrap_psi<1>), grid1(total), dim3(256), 0, s, io, C->st, mixed,
                               wf, total, C->p.dt);
        else
            hipLaunchKernelGGL((k_wrap_psi<2>), grid1(total), dim3(256), 0, s, io, C->st, mixed,
                               wf, total, C->p.dt);
        return;
    }
    const unsigned rb = red_blocks(total);
    // psi^{k+1}, phi^{k+1}, the optional mu and kappa outputs, and the sums
    // of psi^{k+1} and mu (acc[8], acc[9])
    auto k1 = C->p.scheme == 1 ? k_wrap_psi_sums<1, NT> : k_wrap_psi_sums<2, NT>;
    hipLaunchKernelGGL(k1, dim3(rb), dim3(NT), 0, s, io, C->st, mixed, wf, warm ? 1 : 0, total,
                       C->p.dt, C->part, C->pst);
    hipLaunchKernelGGL((k_wrap_partials<NT>), dim3(1), dim3(NT), 0, s, C->st, C->part, (int)rb, 2,
                       C->acc + 8);
    if (!warm) {
        hipLaunchKernelGGL(k_wrap_w_zero, grid1(total), dim3(256), 0, s, C->st, F0.w[0], total);
    } else {
        const double sb = C->p.dt * C->p.beta, sM = C->p.dt * C->p.M;
        double a, b;
        if (C->p.scheme == 1) { a = 1.0 / (1.0 + sb); b = sM / (1.0 + sb); }
        else { a = (1.0 - 0.5 * sb) / (1.0 + 0.5 * sb); b = sM / (1.0 + 0.5 * sb); }
        hipLaunchKernelGGL(k_wrap_w_advance, grid1(total), dim3(256), 0, s, C->st, mixed,
                           F0.u[0][1], F0.u[1][1], F0.w[0], total, a, b, C->acc + 9);
    }
    // b = psi - mean, its square sum (acc[10]), the warm start's squared
    // residual (acc[11]) and the energy sums with the warm start (acc[0..7])
    hipLaunchKernelGGL((k_wrap_rhs_terms<NT>), dim3(rb), dim3(NT), 0, s, C->st, io, F0.g,
                       1.0 / (F0.h * F0.h), C->acc + 8, F0.pf, warm ? F0.w[0] : nullptr, C->part,
                       (const double*)(C->pinned ? F0.pin : nullptr),
                       (const double*)(C->pinned ? C->phihat : nullptr));
    // the warm start's residual is the first norm of the Poisson solve: it
    // may already meet the test, and the cycles behind it then exit at once
    if (warm)
        hipLaunchKernelGGL((k_wrap_partials_pnorm<NT>), dim3(1), dim3(NT), 0, s, C->st, C->part,
                           (int)rb, C->acc, C->pst, C->phist, kPoissonRel, kPoissonStall,
                           kPoissonMax);
    else
        hipLaunchKernelGGL((k_wrap_partials<NT>), dim3(1), dim3(NT), 0, s, C->st, C->part, (int)rb,
                           12, C->acc);
    for (int k = 0; k < npoisson; ++k) vcycle_poisson(C, s);
    // A warm start with no cycle behind it keeps the sums above (the host runs
    // cycles and the sums again if it fails its test): nothing to enqueue.
    if (!warm || npoisson > 0) enqueue_energy_terms(C, s, warm);
}

// Energy sums of phi^{k+1} with the Poisson cycles' w into acc[0..7], when
// any cycle ran (gated on the step's and the Poisson solve's states).
void enqueue_energy_terms(mpfc_ctx* C, hipStream_t s, bool warm) {
    Level& F0 = C->L[0];
    const unsigned rb = red_blocks((size_t)C->m * C->n);
    hipLaunchKernelGGL((k_wrap_terms<NT>), dim3(rb), dim3(NT), 0, s, C->st, C->pst, warm ? 1 : 0,
                       (const StepIO*)C->io, F0.g, 1.0 / (F0.h * F0.h), F0.pf, F0.w[0], C->part,
                       (const double*)(C->pinned ? F0.pin : nullptr),
                       (const double*)(C->pinned ? C->phihat : nullptr));
    hipLaunchKernelGGL((k_wrap_terms_sum<NT>), dim3(1), dim3(NT), 0, s, C->st, C->pst,
                       warm ? 1 : 0, C->part, (int)rb, C->acc);
}

}  // namespace

// ============================================================================
extern "C" {

void mpfc_default_opts(mpfc_opts* o) {
    if (!o) return;
    o->nu1 = 2; o->nu2 = 2; o->max_cycles = 100;
    o->tol = 1e-10;
    o->precision = MPFC_FP64;
    o->guess = MPFC_GUESS_EXTRAP;
    o->linearization = MPFC_NEWTON;
    o->coarsest = 2;
    o->energy = 1;
    o->diverge = 1e8;
    o->inner_cycles = 3;
    o->coarse_sweeps = 2;
    o->omega = 1.0;
    o->coarse_threshold = 0;
    o->inner_cycles_next = 0;
    o->inner_nu_coarse = 0;
}

int mpfc_validate(int m, int n, const mpfc_params* p, const mpfc_opts* o) {
    return validate(m, n, p, o);
}

int mpfc_version(void) { return MPFC_VERSION; }

const char* mpfc_strerror(int code) {
    switch (code) {
        case MPFC_OK: return "success";
        case MPFC_EINVAL: return "invalid argument";
        case MPFC_ENOTCONVERGED: return "cycle limit reached before the tolerance";
        case MPFC_ENONFINITE: return "non-finite residual";
        case MPFC_EDIVERGED: return "residual diverged";
        case MPFC_ENOMEM: return "device memory allocation failed";
        case MPFC_EHIP: return "HIP runtime error";
        default: return "unknown error";
    }
}

const char* mpfc_last_error(void) { return g_last_error.c_str(); }

int mpfc_prof_enable(mpfc_ctx* C, int what) {
    if (!C || what < 0 || what > 1) return fail(MPFC_EINVAL, "mpfc_prof_enable: bad arguments");
    if (what && !C->ev[0])
        for (int k = 0; k < 4; ++k) HIP_TRY(hipEventCreate(&C->ev[k]));
    C->prof = what;
    return MPFC_OK;
}

int mpfc_tile_shape(mpfc_ctx* C, int level, int which, int* tx, int* ty, int* halo) {
    if (!C) return fail(MPFC_EINVAL, "ctx is NULL");
    if (level < 0 || level >= C->Lp || which < 0 || which >= SH_KINDS)
        return fail(MPFC_EINVAL, "no tiled launch of that level and kind");
    const Level& lv = C->L[level];
    const int H = which == SH_DN || which == SH_DN32 ? round_even(2 * C->o.nu1 + 1)
                  : which == SH_UP ? (level == 0 ? round_even(2 * C->o.nu2 + 1) : 2 * C->o.nu2)
                  : which == SH_UP32 ? 2 * C->o.nu2
                  : which == SH_PDN ? 6 : (level == 0 ? 6 : 4);
    const int k = level_shape(lv, which, H);
    int x = 0, y = 0;
    tile_dims(lv, k, x, y);
    if (tx) *tx = x;
    if (ty) *ty = y;
    if (halo) *halo = kShapes[k].hmax;
    return MPFC_OK;
}

int mpfc_prof_read(mpfc_ctx* C, int which, double* total_ms, long long* launches,
                   long long* cells, int reset) {
    if (!C || !total_ms || !launches || !cells || which < 0 || which > 1)
        return fail(MPFC_EINVAL, "mpfc_prof_read: bad arguments");
    *total_ms = C->prof_ms[which];
    *launches = C->prof_launches[which];
    *cells = (long long)C->m * C->n;
    if (reset) { C->prof_ms[which] = 0.0; C->prof_launches[which] = 0; }
    return MPFC_OK;
}

// Context of one grid; `tune` = false skips the tile autotuner (the batched
// path tunes its own launches).
static int create_ctx(mpfc_ctx** out, int m, int n, const mpfc_params* p, const mpfc_opts* o,
                      void* stream, bool tune) {
    if (!out) return fail(MPFC_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(m, n, p, o);
    if (rc) return rc;
    mpfc_ctx* C = new (std::nothrow) mpfc_ctx();
    if (!C) return fail(MPFC_ENOMEM, "host allocation failed");
    C->m = m; C->n = n; C->p = *p; C->o = *o;
    C->stream = (hipStream_t)stream;
    C->alpha = 1.0 - p->eps;
    scheme_coefficients(p, C->c, C->d);
    const char* ng = std::getenv("MPFC_NO_GRAPH");
    C->use_graph = !(ng && ng[0] == '1');
    C->inner_cycles = o->inner_cycles;
    C->inner_next = o->inner_cycles_next ? o->inner_cycles_next : o->inner_cycles;
    C->gen = !(is_pow2(m) && is_pow2(n));
    const bool mixed = o->precision == MPFC_MIXED;
    // level hierarchy; a general grid tiles every level but its coarsest
    {
        int mm = m, nn = n;
        double h = p->h;
        for (;;) {
            Level lv;
            lv.m = mm; lv.n = nn; lv.h = h; lv.g = make_grid(mm, nn, p->bc);
            const bool last = !coarsen_more(mm, nn, o->coarsest);
            lv.tiled = C->gen ? !last : (long long)mm * nn > persistent_cells(o);
            C->L.push_back(lv);
            if (last) break;
            mm /= 2; nn /= 2; h *= 2.0;
        }
    }
    const int nl = (int)C->L.size();
    C->Lp = nl;
    for (int l = 0; l < nl; ++l)
        if (!C->L[l].tiled) { C->Lp = l; break; }
    // Arena layout in doubles, every piece 256-byte aligned: the same function
    // sizes the arena (base == nullptr) and then assigns the pointers.
    const Level& Lc = C->L[nl - 1];
    // coarsest Poisson solve: dense Green's matrix, or (general grid) the
    // separable eigenbasis V_x, V_y and the inverse eigenvalues
    const size_t nG = C->gen ? (size_t)Lc.m * Lc.m + (size_t)Lc.n * Lc.n + (size_t)Lc.m * Lc.n
                             : (size_t)(Lc.m * Lc.n) * (Lc.m * Lc.n);
    auto layout = [&](double* base) {
        size_t off = 0;
        // Pieces start 256-byte aligned; after each one a gap of 0-15 x 256
        // bytes (varying from piece to piece) keeps fields of equal
        // power-of-two size from starting at the same offset modulo the HBM
        // channel interleave, where same-index accesses to several fields
        // would fall on one channel.
        int piece = 0;
        auto take = [&](size_t cnt) {
            double* r = base ? base + off : nullptr;
            off += (cnt + 31) & ~(size_t)31;
            off += (size_t)32 * ((piece * 7) & 15);
            ++piece;
            return r;
        };
        for (int l = 0; l < nl; ++l) {
            Level& lv = C->L[l];
            const size_t Nl = (size_t)lv.m * lv.n;
            for (int f = 0; f < 3; ++f) {
                lv.u[0][f] = take(Nl);
                // level 0 always has copy 1: mixed precision and the learned
                // guess's candidate use it even when the finest level is untiled
                lv.u[1][f] = (l < C->Lp || l == 0) ? take(Nl) : nullptr;
                lv.f[f] = take(Nl);
                lv.v[f] = l > 0 ? take(Nl) : nullptr;
                lv.rr[f] = l > 0 ? take(Nl) : nullptr;
            }
            lv.xk = (p->scheme == 2) ? take(Nl) : nullptr;
            lv.w[0] = take(Nl);
            lv.w[1] = (l < C->Lp) ? take(Nl) : nullptr;
            lv.pf = take(Nl);
            lv.pv = l > 0 ? take(Nl) : nullptr;
            lv.prr = l > 0 ? take(Nl) : nullptr;
        }
        C->phik = C->L[0].xk ? C->L[0].xk : take((size_t)m * n);
        if (mixed) {
            auto take_f = [&](size_t cnt) { return (float*)take((cnt + 1) / 2); };
            C->FL.assign(nl, mpfc_ctx::FLevel{});
            for (int l = 0; l < nl; ++l) {
                auto& F = C->FL[l];
                const size_t Nl = (size_t)C->L[l].m * C->L[l].n;
                for (int f = 0; f < 3; ++f) {
                    F.e[0][f] = take_f(Nl);
                    F.e[1][f] = l < C->Lp ? take_f(Nl) : nullptr;
                    F.v[f] = l > 0 ? take_f(Nl) : nullptr;
                    F.f[f] = take_f(Nl);
                    F.rr[f] = l > 0 ? take_f(Nl) : nullptr;
                }
                F.xk = p->scheme == 2 ? take_f(Nl) : nullptr;
                F.pb = take_f(Nl);
            }
        }
        C->G = take(nG);
        C->rb_count = 32 + (size_t)o->max_cycles + 1;
        C->rb = take(C->rb_count + 8);
        C->st = (CycleState*)C->rb;
        C->pst = (CycleState*)(C->rb + 8);
        C->acc = C->rb + 16;
        C->hist = C->rb + 32;
        C->io = (StepIO*)take(8);
        C->phist = take(64);
        // one partial sum per finest tile (general grids: tiles down to 2 x 2),
        // and at least kWrapSums per reduction workgroup
        const size_t cells_per_part = C->gen ? 4 : 256;
        const size_t min_parts = (size_t)kRedBlocks * kWrapSums;
        C->nparts = (int)((size_t)m * n / cells_per_part > min_parts ? (size_t)m * n / cells_per_part
                                                                      : min_parts);
        C->part = take((size_t)C->nparts);
        C->cnn_r2 = take(8);
        C->cnn_counts = (unsigned long long*)take(8);
        return off;
    };
    C->arena_bytes = layout(nullptr) * sizeof(double);
    hipError_t e = hipMalloc(&C->arena, C->arena_bytes);
    if (e != hipSuccess) {
        delete C;
        return fail(MPFC_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    layout((double*)C->arena);
    std::vector<double> G;
    if (C->gen) spectral_factors(Lc.m, Lc.n, Lc.h, p->bc, G);
    else green_matrix(Lc.m, Lc.n, Lc.h, p->bc, G);
    e = hipHostMalloc((void**)&C->host_buf, sizeof(double) * (C->rb_count + 64),
                          hipHostMallocDefault);
    // zero the whole arena once (the autotuner runs the tile kernels on it)
    if (e == hipSuccess) e = hipMemsetAsync(C->arena, 0, C->arena_bytes, C->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(C->G, G.data(), nG * sizeof(double), hipMemcpyHostToDevice, C->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(C->stream);
    if (e != hipSuccess) {
        mpfc_destroy(C);
        return fail(MPFC_EHIP, std::string("context setup: ") + hipGetErrorString(e));
    }
    rc = tune ? autotune(C) : MPFC_OK;
    if (rc == MPFC_OK) {
        e = hipStreamSynchronize(C->stream);
        if (e != hipSuccess) rc = fail(MPFC_EHIP, std::string("autotune: ") + hipGetErrorString(e));
    }
    if (rc) {
        mpfc_destroy(C);
        return rc;
    }
    *out = C;
    return MPFC_OK;
}

int mpfc_create(mpfc_ctx** out, int m, int n, const mpfc_params* p, const mpfc_opts* o,
                void* stream) {
    return create_ctx(out, m, n, p, o, stream, true);
}

void mpfc_destroy(mpfc_ctx* C) {
    if (!C) return;
    destroy_graphs(C);
    if (C->cap_stream) (void)hipStreamDestroy(C->cap_stream);
    for (hipEvent_t e : C->ev)
        if (e) (void)hipEventDestroy(e);
    if (C->cnn) cnn_free(C->cnn);
    if (C->pin_mem) (void)hipFree(C->pin_mem);
    if (C->arena) (void)hipFree(C->arena);
    if (C->host_buf) (void)hipHostFree(C->host_buf);
    delete C;
}

int mpfc_step(mpfc_ctx* C, const double* phi_n, const double* phi_nm1, double* psi,
              double* phi_np1, double* mu_out, double* ka_out, mpfc_info* info) {
    if (!C) return fail(MPFC_EINVAL, "ctx is NULL");
    if (!phi_n || !psi || !phi_np1) return fail(MPFC_EINVAL, "phi_n, psi and phi_np1 are required");
    if (phi_np1 == phi_n || phi_np1 == phi_nm1 || phi_np1 == psi)
        return fail(MPFC_EINVAL, "phi_np1 must not alias an input");
    if (psi == phi_n || psi == phi_nm1)
        return fail(MPFC_EINVAL, "psi (updated in place) must not alias phi_n or phi_nm1");
    for (const double* o : {(const double*)mu_out, (const double*)ka_out})
        if (o && (o == phi_n || o == phi_nm1 || o == psi || o == phi_np1))
            return fail(MPFC_EINVAL, "mu and kappa outputs must not alias the other arrays");
    if (mu_out && mu_out == ka_out)
        return fail(MPFC_EINVAL, "mu and kappa outputs must be distinct arrays");
    if (!phi_nm1) phi_nm1 = phi_n;
    if (C->o.guess == MPFC_GUESS_CNN && !C->cnn)
        return fail(MPFC_EINVAL, "guess mode MPFC_GUESS_CNN needs a network (mpfc_cnn_load)");
    hipStream_t s = C->stream;
    Level& F0 = C->L[0];
    const size_t total = (size_t)C->m * C->n;
    const bool mixed = C->o.precision == MPFC_MIXED;
    const bool learned = C->o.guess == MPFC_GUESS_CNN;
    // The caller's arrays, for the captured set-up and wrap-up.
    hipLaunchKernelGGL(k_set_io, dim3(1), dim3(64), 0, s, C->io, phi_n, phi_nm1, psi, phi_np1,
                       mu_out, ka_out);
    int rc = run_unit(C, graph_key(GK_PROLOGUE), [&](hipStream_t cs) {
        (void)step_prologue(C, cs);
    });
    if (rc) return rc;
    const CycleState* hst = (const CycleState*)C->host_buf;
    const CycleState* hpst = (const CycleState*)(C->host_buf + 8);
    auto readback = [&](size_t count) -> int {
        HIP_TRY(hipMemcpyAsync(C->host_buf, C->rb, count * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return MPFC_OK;
    };
    const bool warm = C->have_w != 0;
    const int npoisson = C->poisson_cycles;
    auto wrapup = [&]() {
        return run_unit(C, graph_key(GK_WRAPUP, warm ? 1 : 0, npoisson),
                        [&](hipStream_t cs) { enqueue_wrapup(C, cs, warm, npoisson); });
    };
    // Cycles (or mixed-precision outer iterations) are enqueued without
    // waiting for the set-up: as many as the previous step needed, then the
    // wrap-up, which runs only if they were enough (a steady step costs one
    // host round trip).  A cycle enqueued after the stop flag was raised exits
    // at once in every kernel, so speculation only costs launches, never
    // changes the result.  Otherwise the missing cycles run one by one, each
    // followed by a look at the state, and then the wrap-up again.  While
    // profiling, every cycle is waited for, so that each timed launch belongs
    // to a cycle that ran.
    int launched = 0;
    auto one_more = [&]() -> int {
        if (launched > C->o.max_cycles + 1)
            return fail(MPFC_EHIP, "internal: cycle state did not advance");
        int r = run_cycles(C, launched, 1);
        ++launched;
        if (!r) r = readback(8);
        if (!r && C->prof && C->Lp > 0 && !mixed) prof_collect(C);
        return r;
    };
    if (C->prof) {
        rc = readback(8);
        while (!rc && !hst->done) rc = one_more();
        if (!rc) rc = wrapup();
        if (!rc) rc = readback(C->rb_count);
    } else {
        const int batch = C->pred_units < 1 ? 1
                          : (C->pred_units > C->o.max_cycles ? C->o.max_cycles : C->pred_units);
        rc = run_cycles(C, 0, batch);
        launched = batch;
        if (!rc) rc = wrapup();
        if (!rc) rc = readback(C->rb_count);
        if (!rc && !hst->done) {
            while (!rc && !hst->done) rc = one_more();
            if (!rc) rc = wrapup();
            if (!rc) rc = readback(C->rb_count);
        }
    }
    if (rc) return rc;
    // Energies: more Poisson cycles when the ones enqueued up front were not
    // enough, then the sums once more.
    int energy_status = MPFC_OK;
    double en[4] = {0, 0, 0, 0};
    if (C->o.energy) {
        int np = npoisson;
        while (!hpst->done && np < kPoissonMax) {
            for (int k = 0; k < 2; ++k, ++np) {
                rc = run_poisson_cycle(C);
                if (rc) return rc;
            }
            enqueue_energy_terms(C, s, warm);
            HIP_TRY(hipGetLastError());
            rc = readback(32);
            if (rc) return rc;
        }
        if (hpst->status != ST_CONVERGED) energy_status = MPFC_ENOTCONVERGED;
        adapt_poisson_cycles(C, *hpst, warm);
        C->have_w = 1;
        energies_from_sums(C, C->host_buf + 16, en);
    }
    const CycleState fin = *hst;
    const int nouter = fin.count - 1;
    const int ncyc = mixed ? inner_cycles_run(C, nouter) : nouter;
    C->pred_units = nouter > 0 ? nouter : 1;
    const int st_rc = status_code(fin.status);
    if (info) {
        info->n_cycles = ncyc;
        info->status = st_rc;
        info->outer_iters = mixed ? nouter : 0;
        info->energy_status = energy_status;
        info->energy_F = en[0];
        info->energy_pseudo = en[1];
        info->energy_mod = en[2];
        info->mass = en[3];
        const double* hb = C->host_buf + 32;
        info->residual = hb[fin.count - 1];
        if (info->residual_history)
            std::memcpy(info->residual_history, hb, sizeof(double) * fin.count);
    }
    if (st_rc) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "step stopped with status %d after %d cycles", fin.status,
                      ncyc);
        return fail(st_rc, buf);
    }
    return MPFC_OK;
}

int mpfc_set_pinning(mpfc_ctx* C, const double* weight, const double* phihat) {
    if (!C) return fail(MPFC_EINVAL, "ctx is NULL");
    if (weight && !phihat) return fail(MPFC_EINVAL, "pinning needs phi_hat");
    if (weight && (C->p.scheme != 2 || C->o.precision != MPFC_FP64 ||
                   C->o.linearization != MPFC_NEWTON))
        return fail(MPFC_EINVAL,
                    "pinning needs the second-order scheme, FP64 and Newton linearisation");
    hipStream_t s = C->stream;
    // the captured set-up, cycles and wrap-up change (other operator
    // instantiation, pinning terms): capture again
    HIP_TRY(hipStreamSynchronize(s));
    destroy_graphs(C);
    if (!weight) {
        C->pinned = false;
        return MPFC_OK;
    }
    const int nl = (int)C->L.size();
    if (!C->pin_mem) {
        size_t cells = 0;
        for (const Level& lv : C->L) cells += (size_t)lv.m * lv.n;
        cells += (size_t)C->m * C->n;  // phi_hat
        HIP_TRY(hipMalloc(&C->pin_mem, cells * sizeof(double)));
        double* p = C->pin_mem;
        for (Level& lv : C->L) { lv.pin = p; p += (size_t)lv.m * lv.n; }
        C->phihat = p;
    }
    const size_t N = (size_t)C->m * C->n;
    HIP_TRY(hipMemcpyAsync(C->L[0].pin, weight, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(C->phihat, phihat, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    // coarse weights: 2x2 averages, level by level
    for (int l = 1; l < nl; ++l)
        hipLaunchKernelGGL((k_restrict<double, double>), grid2(C->L[l].m, C->L[l].n), B2, 0, s,
                           C->L[l - 1].g, C->L[l - 1].pin, C->L[l].pin);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    C->pinned = true;
    return MPFC_OK;
}

int mpfc_energies(mpfc_ctx* C, const double* phi, const double* phi_prev, const double* psi,
                  double* out) {
    if (!C || !phi || !psi || !out) return fail(MPFC_EINVAL, "ctx, phi, psi and out are required");
    return compute_energies(C, phi, phi_prev, psi, out);
}

// ---- operator-level entry points --------------------------------------------
// Red-black sweeps through the same fused tile kernel the V-cycle uses (down
// direction without the restriction outputs); a scratch copy keeps the
// ping-pong between launches.
}  // extern "C"

namespace {

int op_smooth_check(const mpfc_params* p, int linearization, int m, int n, const double* phik,
                    const double* phi, const double* mu, const double* ka, const double* f1,
                    const double* f2, const double* f3, int sweeps, const char* name) {
    int rc = validate_params(p);
    if (rc) return rc;
    if (m < 4 || n < 4 || (m & 1) || (n & 1) || sweeps < 0 || !phi || !mu || !ka || !f1 ||
        !f2 || !f3 || (p->scheme == 2 && !phik) ||
        !(linearization == MPFC_NEWTON || linearization == MPFC_PICARD))
        return fail(MPFC_EINVAL, std::string(name) + ": bad arguments");
    return MPFC_OK;
}

// Doubles of scratch the sweeps need: a copy of u (3 m n) and one (m/2)(n/2)
// array that takes the down launch's restriction outputs, which are discarded.
size_t op_smooth_scratch(int m, int n) {
    const size_t N = (size_t)m * n;
    return 3 * N + N / 4 + 1;
}

// The passes, with `tmp` (op_smooth_scratch(m, n) doubles of device memory)
// as scratch; ends with a wait on the stream.
int op_smooth_run(const mpfc_params* p, int linearization, int m, int n, const double* phik,
                  double* phi, double* mu, double* ka, const double* f1, const double* f2,
                  const double* f3, int sweeps, hipStream_t s, double* tmp) {
    const size_t N = (size_t)m * n;
    double* cz = tmp + 3 * N;  // coarse outputs land here and are discarded
    double* a[3] = {phi, mu, ka};
    double* b[3] = {tmp, tmp + N, tmp + 2 * N};
    const LevelOp<double> lop = params_op(p);
    Level lv;
    lv.m = m; lv.n = n; lv.g = make_grid(m, n, p->bc);
    int done = 0;
    while (done < sweeps) {
        const int k = (sweeps - done) >= 2 ? 2 : 1;
        TileArgs<double> T{};
        T.g = lv.g;
        for (int f = 0; f < 3; ++f) {
            T.uin[f] = a[f]; T.uout[f] = b[f];
            T.uH[f] = cz; T.vH[f] = cz; T.rH[f] = cz;
        }
        T.f[0] = f1; T.f[1] = f2; T.f[2] = f3;
        T.xk = phik;
        T.nsweep = 2 * k;
        T.H = round_even(2 * k + 1);
        T.complete_f = 0;
        T.norm = 0;
        tile_dims(lv, 0, T.tx, T.ty);
        if (p->scheme == 1) {
            MpfcOp<double, 1, true, false> on{lop};
            MpfcOp<double, 1, false, false> op{lop};
            if (linearization == MPFC_NEWTON) launch_tile<decltype(on), false>(on, T, 0, nullptr, s);
            else launch_tile<decltype(op), false>(op, T, 0, nullptr, s);
        } else {
            MpfcOp<double, 2, true, false> on{lop};
            MpfcOp<double, 2, false, false> op{lop};
            if (linearization == MPFC_NEWTON) launch_tile<decltype(on), false>(on, T, 0, nullptr, s);
            else launch_tile<decltype(op), false>(op, T, 0, nullptr, s);
        }
        for (int f = 0; f < 3; ++f) { double* t = a[f]; a[f] = b[f]; b[f] = t; }
        done += k;
    }
    if (a[0] != phi)
        for (int f = 0; f < 3; ++f) {
            double* dst = f == 0 ? phi : (f == 1 ? mu : ka);
            HIP_TRY(hipMemcpyAsync(dst, a[f], N * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return MPFC_OK;
}

}  // namespace

extern "C" {

int mpfc_op_smooth(const mpfc_params* p, int linearization, int m, int n, const double* phik,
                   double* phi, double* mu, double* ka, const double* f1, const double* f2,
                   const double* f3, int sweeps, void* stream) {
    int rc = op_smooth_check(p, linearization, m, n, phik, phi, mu, ka, f1, f2, f3, sweeps,
                             "mpfc_op_smooth");
    if (rc) return rc;
    double* tmp = nullptr;
    HIP_TRY(hipMalloc(&tmp, op_smooth_scratch(m, n) * sizeof(double)));
    rc = op_smooth_run(p, linearization, m, n, phik, phi, mu, ka, f1, f2, f3, sweeps,
                       (hipStream_t)stream, tmp);
    const hipError_t fe = hipFree(tmp);
    if (rc) return rc;
    if (fe != hipSuccess) return fail(MPFC_EHIP, std::string("hipFree: ") + hipGetErrorString(fe));
    return MPFC_OK;
}

}  // extern "C"

// ---- the same sweeps without allocation ---------------------------------------
// For callers that cannot allocate device memory during a call (code under
// HIP graph capture, tight serving loops): the scratch of mpfc_op_smooth lives
// in a file-scope device array sized for grids of up to kNoAllocMaxCells
// cells.  Each GPU holds its own copy for the life of the process; host code
// uses its device address, looked up once per device, never the name.
namespace {
constexpr int kNoAllocMaxCells = 1 << 18;  // 512 x 512
constexpr size_t kNoAllocScratch = 3 * (size_t)kNoAllocMaxCells + kNoAllocMaxCells / 4 + 1;
}  // namespace

static __device__ __align__(256) double scratch[kNoAllocScratch];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on first use
// with that device current).
int scratch_on_device(double** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MPFC_EHIP, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = (double*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return MPFC_OK;
}
}  // namespace

extern "C" {

int mpfc_op_smooth_noalloc(const mpfc_params* p, int linearization, int m, int n,
                           const double* phik, double* phi, double* mu, double* ka,
                           const double* f1, const double* f2, const double* f3, int sweeps,
                           void* stream) {
    int rc = op_smooth_check(p, linearization, m, n, phik, phi, mu, ka, f1, f2, f3, sweeps,
                             "mpfc_op_smooth_noalloc");
    if (rc) return rc;
    if ((long long)m * n > kNoAllocMaxCells)
        return fail(MPFC_EINVAL, "mpfc_op_smooth_noalloc: more than 512 x 512 cells (the size of "
                                 "its static scratch)");
    static_assert(kNoAllocScratch >= 3 * (size_t)kNoAllocMaxCells + kNoAllocMaxCells / 4 + 1,
                  "the static scratch holds op_smooth_scratch() of the largest grid");
    double* tmp = nullptr;
    rc = scratch_on_device(&tmp);
    if (rc) return rc;
    return op_smooth_run(p, linearization, m, n, phik, phi, mu, ka, f1, f2, f3, sweeps,
                         (hipStream_t)stream, tmp);
}

int mpfc_op_residual(const mpfc_params* p, int m, int n, const double* phik, const double* phi,
                     const double* mu, const double* ka, const double* f1, const double* f2,
                     const double* f3, double* r1, double* r2, double* r3, void* stream) {
    int rc = validate_params(p);
    if (rc) return rc;
    if (m < 2 || n < 2 || (m & 1) || (n & 1) || !phi || !mu || !ka || !f1 || !f2 || !f3 ||
        !r1 || !r2 || !r3 || (p->scheme == 2 && !phik))
        return fail(MPFC_EINVAL, "mpfc_op_residual: bad arguments");
    Fields<double> F;
    F.phi = const_cast<double*>(phi); F.mu = const_cast<double*>(mu); F.ka = const_cast<double*>(ka);
    F.f1 = f1; F.f2 = f2; F.f3 = f3; F.phik = phik; F.base = nullptr;
    const LevelOp<double> op = params_op(p);
    const Grid g = make_grid(m, n, p->bc);
    hipStream_t s = (hipStream_t)stream;
    if (p->scheme == 1)
        hipLaunchKernelGGL((k_residual_field<double, 1, false>), grid2(m, n), B2, 0, s, F, op, g,
                           r1, r2, r3);
    else
        hipLaunchKernelGGL((k_residual_field<double, 2, false>), grid2(m, n), B2, 0, s, F, op, g,
                           r1, r2, r3);
    HIP_TRY(hipGetLastError());
    return MPFC_OK;
}

int mpfc_op_source(const mpfc_params* p, int m, int n, const double* phik, const double* phikm1,
                   const double* psik, double* S1, double* S2, double* S3, void* stream) {
    int rc = validate_params(p);
    if (rc) return rc;
    if (m < 2 || n < 2 || (m & 1) || (n & 1) || !phik || !psik || !S1 || !S2 || !S3)
        return fail(MPFC_EINVAL, "mpfc_op_source: bad arguments");
    if (!phikm1) phikm1 = phik;
    double c, d;
    scheme_coefficients(p, c, d);
    const Grid g = make_grid(m, n, p->bc);
    hipStream_t s = (hipStream_t)stream;
    if (p->scheme == 1)
        hipLaunchKernelGGL((k_source<1>), grid2(m, n), B2, 0, s, g, 1.0 / (p->h * p->h), d,
                           1.0 - p->eps, phik, phikm1, psik, S1, S2, S3, nullptr,
                           (const double*)nullptr, (const double*)nullptr);
    else
        hipLaunchKernelGGL((k_source<2>), grid2(m, n), B2, 0, s, g, 1.0 / (p->h * p->h), d,
                           1.0 - p->eps, phik, phikm1, psik, S1, S2, S3, nullptr,
                           (const double*)nullptr, (const double*)nullptr);
    HIP_TRY(hipGetLastError());
    return MPFC_OK;
}

int mpfc_op_restrict(int m, int n, const double* fine, double* coarse, void* stream) {
    if (m < 2 || n < 2 || (m & 1) || (n & 1) || !fine || !coarse)
        return fail(MPFC_EINVAL, "mpfc_op_restrict: bad arguments");
    hipLaunchKernelGGL((k_restrict<double, double>), grid2(m / 2, n / 2), B2, 0,
                       (hipStream_t)stream, make_grid(m, n, 0), fine, coarse);
    HIP_TRY(hipGetLastError());
    return MPFC_OK;
}

}  // extern "C"

#include "batch_host.hpp"
#include "cnn_host.hpp"
#include "mpfc3d_host.hpp"
