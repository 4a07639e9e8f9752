// Host side of the batched time step (included at the end of mpfc.hip, after
// the single-grid context and its helpers).
//
// A batch is a set of independent simulations, each an internal single-grid
// context (own arena, levels and parameters), advanced by shared launches:
//  - cell phases (set-up, completion, residual/defect, psi update): one launch
//    over the chunks of every simulation's finest grid;
//  - tile phases: the tiled levels of all simulations, grouped by level size
//    (a group holds every simulation's level of that size); down phases run
//    from the largest size to the smallest, up phases the other way, so each
//    simulation sees its own levels in V-cycle order;
//  - one persistent launch with a workgroup per simulation for the coarse
//    levels (phi^k and the base phi of the coarse levels are averaged by the
//    down launches, as in the single-grid path).
// The tile shape of every (size, down/up) phase is chosen by timing each
// shape on the phase's whole work list.  The step's units (set-up, one
// V-cycle or one outer iteration, wrap-up) are captured once as hipGraphs and
// replayed; the caller's buffers reach them through a device table that is
// rewritten before each step.
#pragma once
#include <algorithm>

#include "batch.hpp"

struct mpfc_batch;

namespace {

template <class Op>
struct KindTable {
    int shape = -1;
    BatchTile<Op>* d_args = nullptr;
    BatchItem* d_items = nullptr;
    int nitems = 0;
    int cap_items = 0;
};

struct PhaseKey {
    int m, n;
    std::vector<std::pair<int, int>> members;  // (simulation, level)
};

struct BatchBase {
    virtual ~BatchBase() {}
    virtual int build() = 0;
    virtual int autotune() = 0;
    virtual void prologue(hipStream_t s) = 0;
    virtual void cycle(hipStream_t s) = 0;
    virtual void outer(int from, int ncyc, hipStream_t s) = 0;
    virtual void epilogue(hipStream_t s) = 0;
};

}  // namespace

struct mpfc_batch {
    int nsim = 0;
    mpfc_opts o{};
    int scheme = 2;
    bool mixed = false;
    bool neu = false;        // some member has a Neumann axis
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    std::vector<mpfc_ctx*> C;
    std::vector<void*> allocs;           // device allocations owned by the batch
    std::vector<BSim> hsims;
    BSim* d_sims = nullptr;
    BIo* d_io = nullptr;
    BIo* h_io = nullptr;                 // pinned
    CycleState* d_st = nullptr;          // one state per simulation, contiguous
    CycleState* h_st = nullptr;          // pinned readback
    BatchItem* d_cells = nullptr;
    int ncells = 0;
    std::vector<PhaseKey> phases;        // tile phases, largest size first
    BatchBase* impl = nullptr;
    hipGraphExec_t gx_pro = nullptr, gx_cyc = nullptr, gx_epi = nullptr, gx_out[3] = {};  // outer iterations from copy 0, 1; the step's first
    bool use_graph = true;
    int pred_units = 4;

    template <typename T>
    int dalloc(T** p, size_t count) {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, count * sizeof(T) + 64);
        if (e != hipSuccess) return fail(MPFC_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        allocs.push_back(q);
        *p = (T*)q;
        return MPFC_OK;
    }
};

namespace {

template <int S, bool NW>
struct BatchImpl : BatchBase {
    using Op64 = MpfcOp<double, S, NW, false>;
    using Op32 = MpfcOp<float, S, NW, true>;
    enum { DN64 = 0, UP64 = 1, DN32 = 2, UP32 = 3 };

    mpfc_batch* B;
    std::vector<KindTable<Op64>> t64[2];   // per phase: down, up
    std::vector<KindTable<Op32>> t32[2];
    BatchCoarse<Op64>* d_c64[2] = {};      // persistent tables (coarsest 4 / 8 cells)
    BatchCoarse<Op32>* d_c32[2] = {};
    int nc[2] = {0, 0};

    explicit BatchImpl(mpfc_batch* b) : B(b) {}

    bool fp64() const { return !B->mixed; }

    // Halo of every member of phase p for launch kind `up` (FP64 and FP32 alike).
    int phase_h(int p, int up) const {
        int H = 0;
        for (auto& mb : B->phases[p].members) {
            // FP64 finest up also forms the residual: one more ring of halo
            const bool norm_ring = up && mb.second == 0 && !B->mixed;
            const int h = up ? (norm_ring ? round_even(2 * B->o.nu2 + 1) : 2 * B->o.nu2)
                             : round_even(2 * B->o.nu1 + 1);
            H = h > H ? h : H;
        }
        return H;
    }

    // Fill and upload the table of phase p, kind (precision, up) for `shape`.
    // with_stop = false: no stop flags, no norm (timing runs of the autotuner).
    template <class Op, bool UP, bool F64>
    int fill(KindTable<Op>& kt, int p, int shape, bool with_stop) {
        std::vector<BatchTile<Op>> args;
        std::vector<BatchItem> items;
        const auto& ph = B->phases[p];
        for (int k = 0; k < (int)ph.members.size(); ++k) {
            const int s = ph.members[k].first, l = ph.members[k].second;
            const mpfc_ctx* C = B->C[s];
            const Level& lv = C->L[l];
            BatchTile<Op> bt{};
            if constexpr (F64) {
                bt.op = make_op<Op>(C, lv);
                bt.A = UP ? up_args64(C, l, l == 0 && with_stop) : dn_args64(C, l);
            } else {
                bt.op = make_op32<Op>(C, lv);
                bt.A = UP ? up_args32(C, l) : dn_args32(C, l);
            }
            tile_dims(lv, shape, bt.A.tx, bt.A.ty);
            bt.stop = with_stop ? C->st : nullptr;
            bt.part_off = 0;
            bt.ntx = lv.m / bt.A.tx;
            const int nt = bt.ntx * (lv.n / bt.A.ty);
            for (int t = 0; t < nt; ++t) items.push_back(BatchItem{k, t});
            if (F64 && UP && l == 0) B->hsims[s].ntiles_up = nt;
            args.push_back(bt);
        }
        if (!kt.d_args) {
            int rc = B->dalloc(&kt.d_args, args.size());
            if (rc) return rc;
            // the smallest tile (16 x 16) gives the most items
            size_t cap = 0;
            for (auto& mb : ph.members) {
                const Level& lv = B->C[mb.first]->L[mb.second];
                cap += (size_t)lv.m * lv.n / 256;
            }
            rc = B->dalloc(&kt.d_items, cap);
            if (rc) return rc;
            kt.cap_items = (int)cap;
        }
        if ((int)items.size() > kt.cap_items) return fail(MPFC_EHIP, "internal: batch item overflow");
        HIP_TRY(hipMemcpy(kt.d_args, args.data(), args.size() * sizeof(BatchTile<Op>),
                          hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(kt.d_items, items.data(), items.size() * sizeof(BatchItem),
                          hipMemcpyHostToDevice));
        kt.shape = shape;
        kt.nitems = (int)items.size();
        return MPFC_OK;
    }

    template <class Op, bool UP>
    void launch(const KindTable<Op>& kt, hipStream_t s) {
        if (kt.nitems > 0) launch_tile_batched<Op, UP>(B->neu, kt.shape, kt.d_args, kt.d_items, kt.nitems, s);
    }

    int build() override {
        const int np = (int)B->phases.size();
        for (int up = 0; up < 2; ++up) {
            t64[up].resize(np);
            t32[up].resize(np);
        }
        for (int p = 0; p < np; ++p)
            for (int up = 0; up < 2; ++up) {
                const int sh = pick_shape(phase_h(p, up));
                int rc = 0;
                if (fp64()) rc = up ? fill<Op64, true, true>(t64[1][p], p, sh, true)
                                    : fill<Op64, false, true>(t64[0][p], p, sh, true);
                else rc = up ? fill<Op32, true, false>(t32[1][p], p, sh, true)
                             : fill<Op32, false, false>(t32[0][p], p, sh, true);
                if (rc) return rc;
            }
        // persistent launch tables, grouped by coarsest-grid size
        for (int g = 0; g < 2; ++g) {
            std::vector<BatchCoarse<Op64>> a64;
            std::vector<BatchCoarse<Op32>> a32;
            for (int s = 0; s < B->nsim; ++s) {
                const mpfc_ctx* C = B->C[s];
                if (coarsest_is_4(C) != (g == 0)) continue;
                const Level& top = C->L[C->Lp];
                if (fp64()) a64.push_back(BatchCoarse<Op64>{make_op<Op64>(C, top), coarse_args64(C), C->st});
                else a32.push_back(BatchCoarse<Op32>{make_op32<Op32>(C, top), coarse_args32(C), C->st});
            }
            nc[g] = fp64() ? (int)a64.size() : (int)a32.size();
            if (!nc[g]) continue;
            int rc = fp64() ? B->dalloc(&d_c64[g], a64.size()) : B->dalloc(&d_c32[g], a32.size());
            if (rc) return rc;
            if (fp64())
                HIP_TRY(hipMemcpy(d_c64[g], a64.data(), a64.size() * sizeof(a64[0]), hipMemcpyHostToDevice));
            else
                HIP_TRY(hipMemcpy(d_c32[g], a32.data(), a32.size() * sizeof(a32[0]), hipMemcpyHostToDevice));
        }
        return MPFC_OK;
    }

    // Time every admissible shape of every (phase, down/up) on its whole work
    // list, from a graph; keep the fastest.  MPFC_TILE_SHAPE=<k> forces shape k.
    int autotune() override {
        const char* forced = std::getenv("MPFC_TILE_SHAPE");
        const int np = (int)B->phases.size();
        hipStream_t s = B->stream;
        int rc = MPFC_OK;
        for (int p = 0; p < np && !rc; ++p)
            for (int up = 0; up < 2 && !rc; ++up) {
                const int H = phase_h(p, up);
                auto run_shape = [&](int k, bool timed, float& ms) -> int {
                    int r;
                    if (fp64()) r = up ? fill<Op64, true, true>(t64[1][p], p, k, !timed)
                                       : fill<Op64, false, true>(t64[0][p], p, k, !timed);
                    else r = up ? fill<Op32, true, false>(t32[1][p], p, k, !timed)
                                : fill<Op32, false, false>(t32[0][p], p, k, !timed);
                    if (r || !timed) return r;
                    auto go = [&](hipStream_t st) {
                        if (fp64()) { if (up) launch<Op64, true>(t64[1][p], st); else launch<Op64, false>(t64[0][p], st); }
                        else { if (up) launch<Op32, true>(t32[1][p], st); else launch<Op32, false>(t32[0][p], st); }
                    };
                    return time_in_graph(B->cap_stream, s, kTuneReps, go, ms);
                };
                int best = pick_shape(H);
                if (forced && forced[0]) {
                    const int k = std::atoi(forced);
                    if (k < 0 || k >= kNumShapes) { rc = fail(MPFC_EINVAL, "MPFC_TILE_SHAPE out of range"); break; }
                    if (H <= kShapes[k].hmax) best = k;
                } else {
                    float t[kNumShapes];
                    float best_ms = 1e30f;
                    for (int k = 0; k < kNumShapes && !rc; ++k) {
                        t[k] = 1e30f;
                        if (H > kShapes[k].hmax) continue;
                        rc = run_shape(k, true, t[k]);
                        best_ms = t[k] < best_ms ? t[k] : best_ms;
                    }
                    if (!rc) best = pick_tuned(t, best_ms, H);
                }
                float dummy = 0.f;
                if (!rc) rc = run_shape(best, false, dummy);
            }
        return rc;
    }

    void finalize(int tiles, hipStream_t s) {
        hipLaunchKernelGGL((k_b_finalize<NT>), dim3(B->nsim), dim3(NT), 0, s, B->d_sims, tiles,
                           B->o.tol, B->o.max_cycles + 1, B->o.diverge);
    }

    void prologue(hipStream_t s) override {
        hipLaunchKernelGGL(k_b_state_reset, dim3((B->nsim + 63) / 64), dim3(64), 0, s, B->d_sims,
                           B->nsim);
        const dim3 gc(B->ncells), blk(256);
        const int mode = B->o.guess == MPFC_GUESS_EXTRAP ? 1 : 0;
        hipLaunchKernelGGL((k_b_setup<S>), gc, blk, 0, s, B->d_sims, B->d_io, B->d_cells, mode);
        hipLaunchKernelGGL(k_b_kappa, gc, blk, 0, s, B->d_sims, B->d_cells);
        if (B->mixed) {
            hipLaunchKernelGGL((k_b_mu<S, true>), gc, blk, 0, s, B->d_sims, B->d_cells);
            hipLaunchKernelGGL((k_b_defect<S>), gc, blk, 0, s, B->d_sims, B->d_cells, 0, 0);
        } else {
            hipLaunchKernelGGL((k_b_mu<S, false>), gc, blk, 0, s, B->d_sims, B->d_cells);
            hipLaunchKernelGGL((k_b_resnorm<S>), gc, blk, 0, s, B->d_sims, B->d_cells);
        }
        finalize(0, s);
    }

    // One FAS V-cycle of every simulation (FP64).
    void cycle(hipStream_t s) override {
        const int np = (int)B->phases.size();
        for (int p = 0; p < np; ++p) launch<Op64, false>(t64[0][p], s);
        if (nc[0]) launch_coarse_batched<Op64, 4>(B->neu, nc[0], d_c64[0], s);
        if (nc[1]) launch_coarse_batched<Op64, 8>(B->neu, nc[1], d_c64[1], s);
        for (int p = np - 1; p >= 0; --p) launch<Op64, true>(t64[1][p], s);
        finalize(1, s);
    }

    // One outer iteration of mixed precision from FP64 copy `from` with
    // `ncyc` FP32 cycles.
    void outer(int from, int ncyc, hipStream_t s) override {
        const int np = (int)B->phases.size();
        hipLaunchKernelGGL(k_b_clear_e, dim3(B->ncells), dim3(256), 0, s, B->d_sims, B->d_cells);
        for (int k = 0; k < ncyc; ++k) {
            for (int p = 0; p < np; ++p) launch<Op32, false>(t32[0][p], s);
            if (nc[0]) launch_coarse_batched<Op32, 4>(B->neu, nc[0], d_c32[0], s);
            if (nc[1]) launch_coarse_batched<Op32, 8>(B->neu, nc[1], d_c32[1], s);
            for (int p = np - 1; p >= 0; --p) launch<Op32, true>(t32[1][p], s);
        }
        hipLaunchKernelGGL((k_b_defect<S>), dim3(B->ncells), dim3(256), 0, s, B->d_sims,
                           B->d_cells, from, 1);
        finalize(0, s);
    }

    void epilogue(hipStream_t s) override {
        if (B->mixed)
            hipLaunchKernelGGL((k_b_psi<S, true>), dim3(B->ncells), dim3(256), 0, s, B->d_sims,
                               B->d_io, B->d_cells);
        else
            hipLaunchKernelGGL((k_b_psi<S, false>), dim3(B->ncells), dim3(256), 0, s, B->d_sims,
                               B->d_io, B->d_cells);
    }
};

enum BatchUnit { BU_PRO = 0, BU_CYC = 1, BU_OUT0 = 2, BU_OUT1 = 3, BU_OUTF = 4, BU_EPI = 5 };

// FP32 cycles of the later outer iterations of a step (inner_cycles_next, 0: inner_cycles).
int batch_inner_next(const mpfc_batch* B) {
    return B->o.inner_cycles_next ? B->o.inner_cycles_next : B->o.inner_cycles;
}

void batch_enqueue(mpfc_batch* B, int unit, hipStream_t s) {
    switch (unit) {
        case BU_PRO: B->impl->prologue(s); break;
        case BU_CYC: B->impl->cycle(s); break;
        case BU_OUT0: B->impl->outer(0, batch_inner_next(B), s); break;
        case BU_OUT1: B->impl->outer(1, batch_inner_next(B), s); break;
        case BU_OUTF: B->impl->outer(1, B->o.inner_cycles, s); break;
        default: B->impl->epilogue(s); break;
    }
}

// Replay a unit from a graph captured on first use (direct launches with
// MPFC_NO_GRAPH=1).
int batch_run(mpfc_batch* B, int unit) {
    hipStream_t s = B->stream;
    if (!B->use_graph) {
        batch_enqueue(B, unit, s);
        HIP_TRY(hipGetLastError());
        return MPFC_OK;
    }
    hipGraphExec_t& gx = unit == BU_PRO ? B->gx_pro
                         : unit == BU_CYC ? B->gx_cyc
                         : unit == BU_EPI ? B->gx_epi
                                          : B->gx_out[unit - BU_OUT0];
    if (!gx) {
        if (!B->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal));
        batch_enqueue(B, unit, B->cap_stream);
        hipError_t le = hipGetLastError();
        hipError_t ce = hipStreamEndCapture(B->cap_stream, &g);
        if (le != hipSuccess || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(MPFC_EHIP, std::string("batch graph capture: ") +
                                       hipGetErrorString(le != hipSuccess ? le : ce));
        }
        hipError_t ie = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            gx = nullptr;
            return fail(MPFC_EHIP, std::string("batch graph instantiate: ") + hipGetErrorString(ie));
        }
    }
    HIP_TRY(hipGraphLaunch(gx, s));
    return MPFC_OK;
}

}  // namespace

extern "C" {

void mpfc_batch_destroy(mpfc_batch* B) {
    if (!B) return;
    if (B->stream) (void)hipStreamSynchronize(B->stream);
    for (hipGraphExec_t g : {B->gx_pro, B->gx_cyc, B->gx_epi, B->gx_out[0], B->gx_out[1], B->gx_out[2]})
        if (g) (void)hipGraphExecDestroy(g);
    if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
    delete B->impl;
    for (void* p : B->allocs) (void)hipFree(p);
    if (B->h_io) (void)hipHostFree(B->h_io);
    if (B->h_st) (void)hipHostFree(B->h_st);
    for (mpfc_ctx* C : B->C) mpfc_destroy(C);
    delete B;
}

int mpfc_batch_create(mpfc_batch** out, int nsim, const mpfc_sim_desc* sims, const mpfc_opts* o,
                      void* stream) {
    if (!out) return fail(MPFC_EINVAL, "out is NULL");
    *out = nullptr;
    if (nsim < 1 || nsim > MPFC_BATCH_MAX) return fail(MPFC_EINVAL, "nsim out of range");
    if (!sims || !o) return fail(MPFC_EINVAL, "sims and opts are required");
    if (o->guess == MPFC_GUESS_CNN)
        return fail(MPFC_EINVAL, "the learned guess is not available in a batch");
    for (int s = 0; s < nsim; ++s) {
        if (!is_pow2(sims[s].m) || !is_pow2(sims[s].n))
            return fail(MPFC_EINVAL, "every simulation of a batch needs power-of-two sides");
        int rc = validate(sims[s].m, sims[s].n, &sims[s].p, o);
        if (rc) {
            char buf[64];
            std::snprintf(buf, sizeof buf, " (simulation %d)", s);
            return fail(rc, g_last_error + buf);
        }
        if (sims[s].p.scheme != sims[0].p.scheme)
            return fail(MPFC_EINVAL, "every simulation of a batch must use the same scheme");
        if ((long long)sims[s].m * sims[s].n <= CP_CELLS)
            return fail(MPFC_EINVAL, "batched grids need more than 1024 cells");
    }
    if (o->coarse_threshold != 0)
        return fail(MPFC_EINVAL, "a batch runs with the default coarse_threshold (0)");
    mpfc_batch* B = new (std::nothrow) mpfc_batch();
    if (!B) return fail(MPFC_ENOMEM, "host allocation failed");
    B->nsim = nsim;
    B->o = *o;
    B->o.energy = 0;
    B->scheme = sims[0].p.scheme;
    B->mixed = o->precision == MPFC_MIXED;
    for (int s = 0; s < nsim; ++s) B->neu = B->neu || sims[s].p.bc != 0;
    B->stream = (hipStream_t)stream;
    const char* ng = std::getenv("MPFC_NO_GRAPH");
    B->use_graph = !(ng && ng[0] == '1');
    int rc = MPFC_OK;
    auto bail = [&](int code) {
        mpfc_batch_destroy(B);
        return code;
    };
    for (int s = 0; s < nsim; ++s) {
        mpfc_ctx* C = nullptr;
        rc = create_ctx(&C, sims[s].m, sims[s].n, &sims[s].p, &B->o, stream, false);
        if (rc) return bail(rc);
        B->C.push_back(C);
    }
    // contiguous cycle states (one readback per check)
    if ((rc = B->dalloc(&B->d_st, nsim))) return bail(rc);
    if (hipMemset(B->d_st, 0, nsim * sizeof(CycleState)) != hipSuccess)
        return bail(fail(MPFC_EHIP, "hipMemset"));
    for (int s = 0; s < nsim; ++s) B->C[s]->st = B->d_st + s;
    if (hipHostMalloc((void**)&B->h_st, nsim * sizeof(CycleState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&B->h_io, nsim * sizeof(BIo), hipHostMallocDefault) != hipSuccess)
        return bail(fail(MPFC_ENOMEM, "hipHostMalloc"));
    // per-simulation records and the cell work list
    std::vector<BatchItem> cells;
    for (int s = 0; s < nsim; ++s) {
        const mpfc_ctx* C = B->C[s];
        const Level& F0 = C->L[0];
        BSim S{};
        S.g = F0.g;
        S.ih2 = 1.0 / (F0.h * F0.h);
        S.h2 = F0.h * F0.h;
        S.d = C->d;
        S.alpha = C->alpha;
        S.al = C->p.scheme == 1 ? C->alpha : 0.5 * C->alpha;
        S.e = C->p.scheme == 1 ? 1.0 : 0.5;
        S.dt = C->p.dt;
        S.op = level_op(C, F0);
        for (int f = 0; f < 3; ++f) {
            S.S[f] = F0.f[f];
            S.u[0][f] = F0.u[0][f];
            S.u[1][f] = F0.u[1][f];
            if (B->mixed) {
                S.fe[f] = C->FL[0].e[0][f];
                S.fr[f] = C->FL[0].f[f];
            }
        }
        S.phik = C->phik;
        if (B->mixed) {
            S.fpb = C->FL[0].pb;
            S.fxk = C->FL[0].xk;
        }
        S.st = C->st;
        S.hist = C->hist;
        S.part = C->part;
        S.nchunks = (int)((size_t)F0.m * F0.n / BCHUNK);
        S.ntiles_up = 0;
        B->hsims.push_back(S);
        for (int c = 0; c < S.nchunks; ++c) cells.push_back(BatchItem{s, c});
    }
    B->ncells = (int)cells.size();
    if ((rc = B->dalloc(&B->d_cells, cells.size()))) return bail(rc);
    if (hipMemcpy(B->d_cells, cells.data(), cells.size() * sizeof(BatchItem), hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(MPFC_EHIP, "hipMemcpy"));
    if ((rc = B->dalloc(&B->d_sims, nsim)) || (rc = B->dalloc(&B->d_io, nsim))) return bail(rc);
    // tile phases: one per distinct tiled level size, largest first
    for (int s = 0; s < nsim; ++s)
        for (int l = 0; l < B->C[s]->Lp; ++l) {
            const Level& lv = B->C[s]->L[l];
            PhaseKey* ph = nullptr;
            for (auto& k : B->phases)
                if (k.m == lv.m && k.n == lv.n) ph = &k;
            if (!ph) {
                B->phases.push_back(PhaseKey{lv.m, lv.n, {}});
                ph = &B->phases.back();
            }
            ph->members.push_back({s, l});
        }
    std::sort(B->phases.begin(), B->phases.end(), [](const PhaseKey& a, const PhaseKey& b) {
        const long long ca = (long long)a.m * a.n, cb = (long long)b.m * b.n;
        return ca != cb ? ca > cb : a.m > b.m;
    });
    const bool nw = o->linearization == MPFC_NEWTON;
    if (B->scheme == 1) B->impl = nw ? (BatchBase*)new BatchImpl<1, true>(B) : new BatchImpl<1, false>(B);
    else B->impl = nw ? (BatchBase*)new BatchImpl<2, true>(B) : new BatchImpl<2, false>(B);
    if ((rc = B->impl->build())) return bail(rc);
    if ((rc = B->impl->autotune())) return bail(rc);
    if (hipMemcpy(B->d_sims, B->hsims.data(), nsim * sizeof(BSim), hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(MPFC_EHIP, "hipMemcpy"));
    if (hipDeviceSynchronize() != hipSuccess) return bail(fail(MPFC_EHIP, "batch set-up"));
    *out = B;
    return MPFC_OK;
}

int mpfc_batch_step(mpfc_batch* B, const double* const* phi_n, const double* const* phi_nm1,
                    double* const* psi, double* const* phi_np1, mpfc_info* infos) {
    if (!B) return fail(MPFC_EINVAL, "batch is NULL");
    if (!phi_n || !psi || !phi_np1) return fail(MPFC_EINVAL, "phi_n, psi and phi_np1 are required");
    for (int s = 0; s < B->nsim; ++s) {
        const double* pn = phi_n[s];
        const double* pm = phi_nm1 && phi_nm1[s] ? phi_nm1[s] : pn;
        if (!pn || !psi[s] || !phi_np1[s]) return fail(MPFC_EINVAL, "NULL buffer in a batch step");
        if (phi_np1[s] == pn || phi_np1[s] == pm || phi_np1[s] == psi[s])
            return fail(MPFC_EINVAL, "phi_np1 must not alias an input");
        B->h_io[s] = BIo{pn, pm, psi[s], phi_np1[s]};
    }
    hipStream_t s = B->stream;
    HIP_TRY(hipMemcpyAsync(B->d_io, B->h_io, B->nsim * sizeof(BIo), hipMemcpyHostToDevice, s));
    int rc = batch_run(B, BU_PRO);
    if (rc) return rc;
    // speculative units (a unit enqueued after a simulation stopped is a no-op for it)
    int launched = 0;
    int batch = B->pred_units > 1 ? B->pred_units - 1 : 1;
    for (;;) {
        if (launched > B->o.max_cycles + 1)
            return fail(MPFC_EHIP, "internal: batch cycle state did not advance");
        for (int k = 0; k < batch; ++k, ++launched) {
            const int unit = !B->mixed ? BU_CYC : launched == 0 ? BU_OUTF : BU_OUT0 + (1 ^ (launched & 1));
            rc = batch_run(B, unit);
            if (rc) return rc;
        }
        batch = 1;
        HIP_TRY(hipMemcpyAsync(B->h_st, B->d_st, B->nsim * sizeof(CycleState),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        bool all = true;
        for (int k = 0; k < B->nsim; ++k) all = all && B->h_st[k].done;
        if (all) break;
    }
    rc = batch_run(B, BU_EPI);
    if (rc) return rc;
    int worst = MPFC_OK, worst_sim = -1, nmax = 1;
    for (int k = 0; k < B->nsim; ++k) {
        const CycleState& st = B->h_st[k];
        const int nouter = st.count - 1;
        nmax = nouter > nmax ? nouter : nmax;
        const int code = status_code(st.status);
        if (code && worst == MPFC_OK) { worst = code; worst_sim = k; }
        if (infos) {
            mpfc_info& I = infos[k];
            I.n_cycles = !B->mixed ? nouter
                         : nouter > 0 ? B->o.inner_cycles + (nouter - 1) * batch_inner_next(B) : 0;
            I.status = code;
            I.outer_iters = B->mixed ? nouter : 0;
            I.energy_status = MPFC_OK;  // a batch computes no energies
            I.energy_F = I.energy_pseudo = I.energy_mod = I.mass = 0.0;
            I.residual = st.acc;
            if (I.residual_history)
                HIP_TRY(hipMemcpyAsync(I.residual_history, B->C[k]->hist,
                                       sizeof(double) * st.count, hipMemcpyDeviceToHost, s));
        }
    }
    B->pred_units = nmax;
    HIP_TRY(hipStreamSynchronize(s));
    if (worst) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "simulation %d stopped with status %d", worst_sim,
                      B->h_st[worst_sim].status);
        return fail(worst, buf);
    }
    return MPFC_OK;
}

int mpfc_batch_size(const mpfc_batch* B) { return B ? B->nsim : 0; }

}  // extern "C"
