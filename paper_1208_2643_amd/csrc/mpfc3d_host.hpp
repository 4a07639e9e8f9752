// Host side of the three-dimensional step (mpfc3d_*): level hierarchy in one
// arena, V-cycles of the MPFC system and of the Poisson problem of the energies
// captured once as HIP graphs and replayed, the stopping test on the device
// (every cycle kernel returns at once after the stop flag is set, so cycles
// can be enqueued ahead of the readback).  Included at the end of mpfc.hip.
#include "mpfc3d.hpp"

namespace {

struct Level3 {
    int m = 0, n = 0, l = 0;
    double h = 0;
    Grid3 g{};
    double* u[3] = {};   // iterate (in place: red-black sweeps update one colour at a time)
    double* f[3] = {};   // right-hand side (finest: S; coarse: completed FAS right-hand side)
    double* v[3] = {};   // restricted iterate (coarse levels)
    double* rr[3] = {};  // restricted residual (coarse levels)
    double* xk = nullptr;
    double* w = nullptr;    // Poisson iterate
    double* pf = nullptr;   // Poisson right-hand side (finest: b = psi - mean)
    double* pv = nullptr;
    double* prr = nullptr;
};

Grid3 make_grid3(int m, int n, int l) { return Grid3{m, n, l, ilog2(m), ilog2(n), ilog2(l)}; }
unsigned blocks256(size_t cells) { return (unsigned)((cells + 255) / 256); }
// Reductions in three dimensions: each workgroup sums one contiguous range,
// whose z-neighbour planes stay in L2 better with 256 long ranges than with
// the 2-D count (measured: the 128^3 residual norm 30 us vs 36 us).
constexpr unsigned kRedBlocks3 = 256;
unsigned red_blocks3(size_t total) {
    const size_t b = (total + NT - 1) / NT;
    return (unsigned)(b < kRedBlocks3 ? b : kRedBlocks3);
}

constexpr int kPoissonCoarseSweeps3 = 10;

int validate3(int m, int n, int l, const mpfc_params* p, const mpfc_opts* o) {
    int rc = validate(4, 4, p, o);  // parameters and options (2-D size rules aside)
    if (rc) return rc;
    if (p->bc != 0) return fail(MPFC_EINVAL, "the three-dimensional step is periodic (bc = 0)");
    if (!is_pow2(m) || !is_pow2(n) || !is_pow2(l) || m < 2 || n < 2 || l < 2)
        return fail(MPFC_EINVAL, "m, n and l must be powers of two >= 2");
    if ((long long)m * n * l > (1LL << 28))
        return fail(MPFC_EINVAL, "grid too large (m*n*l > 2^28)");
    if (o->precision != MPFC_FP64)
        return fail(MPFC_EINVAL, "the three-dimensional step runs in MPFC_FP64");
    if (o->guess == MPFC_GUESS_CNN)
        return fail(MPFC_EINVAL, "the learned guess is two-dimensional");
    if (o->omega != 1.0)
        return fail(MPFC_EINVAL, "the three-dimensional step runs App. B's smoother (omega = 1)");
    if (o->coarse_threshold != 0)
        return fail(MPFC_EINVAL, "the three-dimensional step takes coarse_threshold = 0");
    return MPFC_OK;
}

}  // namespace

struct mpfc3d_ctx {
    int m = 0, n = 0, l = 0;
    mpfc_params p{};
    mpfc_opts o{};
    hipStream_t stream = nullptr;
    double c = 0, d = 0, alpha = 0;
    std::vector<Level3> L;
    int Lp = 0;                         // first level of at most CP3_CELLS cells (persistent kernel)
    CycleState* st = nullptr;
    double* hist = nullptr;
    CycleState* pst = nullptr;
    double* phist = nullptr;
    double* acc = nullptr;
    double* part = nullptr;
    int nparts = 0;
    void* arena = nullptr;
    CycleState* host_st = nullptr;
    double* host_buf = nullptr;
    bool have_w = false;
    int pred = 4;                       // cycles the last step needed
    hipGraphExec_t gx[2] = {};          // one V-cycle: MPFC, Poisson
    hipStream_t cap = nullptr;
    int prof = 0;
    hipEvent_t ev[2] = {};
    double prof_ms = 0;
    long long prof_launches = 0;
};

namespace {

LevelOp<double> level_op3(const mpfc3d_ctx* C, const Level3& lv) {
    LevelOp<double> o;
    o.ih2 = 1.0 / (lv.h * lv.h);
    o.c = C->c;
    o.al = C->p.scheme == 1 ? C->alpha : 0.5 * C->alpha;
    o.e = C->p.scheme == 1 ? 1.0 : 0.5;
    return o;
}

// One red-black half-sweep launch; on the finest level, timed with events
// while profiling (cycles then run without graphs).
template <class Op>
int relax3(mpfc3d_ctx* C, const Op& op, const Level3& lv, const L3& A, int colour,
           const CycleState* stop, hipStream_t s, bool finest) {
    const size_t half = (size_t)lv.m * lv.n * lv.l / 2;
    const bool timed = finest && C->prof;
    if (timed) HIP_TRY(hipEventRecord(C->ev[0], s));
    hipLaunchKernelGGL((k3_relax<Op>), dim3(blocks256(half)), dim3(256), 0, s, op, lv.g, A, colour,
                       stop);
    if (timed) {
        HIP_TRY(hipEventRecord(C->ev[1], s));
        HIP_TRY(hipEventSynchronize(C->ev[1]));
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, C->ev[0], C->ev[1]));
        C->prof_ms += ms;
        C->prof_launches += 1;
    }
    return MPFC_OK;
}

// One FAS V(nu1, nu2) cycle of the MPFC system (or, POISSON, of -Lap w = b),
// then the finest residual norm and the stopping test.
template <class Op, bool POISSON>
int vcycle3(mpfc3d_ctx* C, hipStream_t s) {
    const int nl = (int)C->L.size();
    const CycleState* stop = POISSON ? C->pst : C->st;
    auto op_of = [&](const Level3& lv) {
        if constexpr (POISSON) {
            return PoissonOp3{1.0 / (lv.h * lv.h), lv.h * lv.h};
        } else {
            return Op{level_op3(C, lv)};
        }
    };
    auto fields = [&](const Level3& lv, int lvl) {
        L3 A{};
        if constexpr (POISSON) {
            A.u[0] = lv.w;
            A.f[0] = lv.pf;
        } else {
            for (int f = 0; f < 3; ++f) { A.u[f] = lv.u[f]; A.f[f] = lv.f[f]; }
            A.xk = lv.xk;
        }
        (void)lvl;
        return A;
    };
    const int nu1 = POISSON ? 2 : C->o.nu1, nu2 = POISSON ? 2 : C->o.nu2;
    const int csweeps = POISSON ? kPoissonCoarseSweeps3 : C->o.coarse_sweeps;
    const bool pers = C->Lp < nl;               // small levels in one persistent launch
    const int top = pers ? C->Lp : nl - 1;      // levels below `top` use per-level launches
    for (int lv = 0; lv < top; ++lv) {
        const Level3& A = C->L[lv];
        const Level3& B = C->L[lv + 1];
        const auto op = op_of(A);
        const L3 FA = fields(A, lv);
        for (int k = 0; k < nu1; ++k)
            for (int col = 0; col < 2; ++col) {
                int rc = relax3(C, op, A, FA, col, stop, s, lv == 0);
                if (rc) return rc;
            }
        L3 FB = fields(B, lv + 1);
        const size_t ncB = (size_t)B.m * B.n * B.l;
        if constexpr (POISSON) {
            hipLaunchKernelGGL((k3_restrict<PoissonOp3>), dim3(blocks256(ncB)), dim3(256), 0, s, op,
                               A.g, FA, FB, B.pv, nullptr, nullptr, B.prr, nullptr, nullptr,
                               nullptr, stop);
            L3 FR{};
            FR.u[0] = B.w;
            FR.f[0] = B.prr;
            if (!(pers && lv + 1 == top))
                hipLaunchKernelGGL((k3_complete<PoissonOp3>), dim3(blocks256(ncB)), dim3(256), 0, s,
                                   op_of(B), B.g, FR, B.pf, nullptr, nullptr, stop);
        } else {
            hipLaunchKernelGGL((k3_restrict<Op>), dim3(blocks256(ncB)), dim3(256), 0, s, op, A.g, FA,
                               FB, B.v[0], B.v[1], B.v[2], B.rr[0], B.rr[1], B.rr[2],
                               Op::XK ? B.xk : nullptr, stop);
            L3 FR{};
            for (int f = 0; f < 3; ++f) { FR.u[f] = B.u[f]; FR.f[f] = B.rr[f]; }
            FR.xk = B.xk;
            if (!(pers && lv + 1 == top))
                hipLaunchKernelGGL((k3_complete<Op>), dim3(blocks256(ncB)), dim3(256), 0, s, op_of(B),
                                   B.g, FR, B.f[0], B.f[1], B.f[2], stop);
        }
    }
    if (pers) {
        // levels top .. nl-1 in one workgroup
        const Level3& T = C->L[top];
        CoarseArgs3 CA{};
        CA.geo.nlev = nl - top;
        int off = 0;
        for (int k = 0; k < CA.geo.nlev; ++k) {
            const Level3& lv = C->L[top + k];
            CA.geo.m[k] = lv.m; CA.geo.n[k] = lv.n; CA.geo.l[k] = lv.l;
            CA.geo.lm[k] = lv.g.lm; CA.geo.ln[k] = lv.g.ln;
            CA.geo.off[k] = off;
            off += lv.m * lv.n * lv.l;
        }
        CA.gtop = T.g;
        CA.complete_top = top > 0;
        CA.nsw1 = nu1;
        CA.nsw2 = nu2;
        CA.nswc = csweeps;
        if constexpr (POISSON) {
            CA.u[0] = T.w;
            CA.f[0] = top > 0 ? T.prr : T.pf;
            CA.xk = nullptr;
        } else {
            for (int f = 0; f < 3; ++f) {
                CA.u[f] = T.u[f];
                CA.f[f] = top > 0 ? T.rr[f] : T.f[f];
            }
            CA.xk = T.xk;
        }
        if constexpr (POISSON)
            hipLaunchKernelGGL((k3_coarse<PoissonOp3>), dim3(1), dim3(CP3_THREADS), 0, s, op_of(T), CA,
                               stop);
        else
            hipLaunchKernelGGL((k3_coarse<Op>), dim3(1), dim3(CP3_THREADS), 0, s, op_of(T), CA, stop);
    } else {
        // coarsest level: red-black sweeps
        const Level3& A = C->L[nl - 1];
        const auto op = op_of(A);
        const L3 FA = fields(A, nl - 1);
        for (int k = 0; k < csweeps; ++k)
            for (int col = 0; col < 2; ++col) {
                int rc = relax3(C, op, A, FA, col, stop, s, nl == 1);
                if (rc) return rc;
            }
    }
    for (int lv = top - 1; lv >= 0; --lv) {
        const Level3& A = C->L[lv];
        const Level3& B = C->L[lv + 1];
        const auto op = op_of(A);
        const L3 FA = fields(A, lv);
        const L3 FB = fields(B, lv + 1);
        const size_t nc = (size_t)A.m * A.n * A.l / 2;   // pairs of fine cells
        // blocked prolongation: whole blocks of P3X x P3Y x P3Z pairs (sides
        // are powers of two, so m >= 2 P3X with n, l >= 4 tiles the level)
        const bool blk = A.m >= 2 * P3X && A.n >= P3Y && A.l >= P3Z;
        const size_t ncB = (size_t)B.m * B.n * B.l;
        if constexpr (POISSON) {
            hipLaunchKernelGGL((k3_correction<1>), dim3(blocks256(ncB)), dim3(256), 0, s, B.g, FB,
                               B.pv, (double*)nullptr, (double*)nullptr, stop);
            if (blk)
                hipLaunchKernelGGL((k3_prolong_blk<1>), dim3(blocks256(nc)), dim3(256), 0, s, A.g,
                                   FA, (const double*)B.pv, (const double*)nullptr,
                                   (const double*)nullptr, stop);
            else
                hipLaunchKernelGGL((k3_prolong<1>), dim3(blocks256(nc)), dim3(256), 0, s, A.g, FA,
                                   (const double*)B.pv, (const double*)nullptr,
                                   (const double*)nullptr, stop);
        } else {
            hipLaunchKernelGGL((k3_correction<3>), dim3(blocks256(ncB)), dim3(256), 0, s, B.g, FB,
                               B.v[0], B.v[1], B.v[2], stop);
            if (blk)
                hipLaunchKernelGGL((k3_prolong_blk<3>), dim3(blocks256(nc)), dim3(256), 0, s, A.g,
                                   FA, (const double*)B.v[0], (const double*)B.v[1],
                                   (const double*)B.v[2], stop);
            else
                hipLaunchKernelGGL((k3_prolong<3>), dim3(blocks256(nc)), dim3(256), 0, s, A.g, FA,
                                   (const double*)B.v[0], (const double*)B.v[1],
                                   (const double*)B.v[2], stop);
        }
        for (int k = 0; k < nu2; ++k)
            for (int col = 0; col < 2; ++col) {
                int rc = relax3(C, op, A, FA, col, stop, s, lv == 0);
                if (rc) return rc;
            }
    }
    // finest residual norm and stopping test
    const Level3& F0 = C->L[0];
    const size_t total = (size_t)F0.m * F0.n * F0.l;
    const unsigned nb = red_blocks3(total);
    const L3 FF = fields(F0, 0);
    if constexpr (POISSON) {
        hipLaunchKernelGGL((k3_resnorm<PoissonOp3, NT>), dim3(nb), dim3(NT), 0, s, op_of(F0), F0.g,
                           FF, C->part, stop);
        hipLaunchKernelGGL((k_p_finalize<NT>), dim3(1), dim3(NT), 0, s, C->part, (int)nb, C->pst,
                           C->phist, C->acc + 10, kPoissonRel, kPoissonStall, kPoissonMax);
    } else {
        hipLaunchKernelGGL((k3_resnorm<Op, NT>), dim3(nb), dim3(NT), 0, s, op_of(F0), F0.g, FF,
                           C->part, stop);
        hipLaunchKernelGGL((k_norm_finalize<NT>), dim3(1), dim3(NT), 0, s, C->part, (int)nb, C->st,
                           C->hist, F0.h * F0.h * F0.h, C->o.tol, C->o.max_cycles + 1,
                           C->o.diverge);
    }
    HIP_TRY(hipGetLastError());
    return MPFC_OK;
}

int enqueue3(mpfc3d_ctx* C, int kind, hipStream_t s) {
    if (kind == 1) return vcycle3<PoissonOp3, true>(C, s);
    const bool nw = C->o.linearization == MPFC_NEWTON;
    if (C->p.scheme == 1)
        return nw ? vcycle3<MpfcOp3<1, true>, false>(C, s) : vcycle3<MpfcOp3<1, false>, false>(C, s);
    return nw ? vcycle3<MpfcOp3<2, true>, false>(C, s) : vcycle3<MpfcOp3<2, false>, false>(C, s);
}

// One cycle (kind 0: MPFC, 1: Poisson) from its graph, captured on first use;
// launched directly while profiling.
int run_cycle3(mpfc3d_ctx* C, int kind) {
    if (C->prof) return enqueue3(C, kind, C->stream);
    hipGraphExec_t& gx = C->gx[kind];
    if (!gx) {
        if (!C->cap) HIP_TRY(hipStreamCreateWithFlags(&C->cap, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(C->cap, hipStreamCaptureModeThreadLocal));
        int rc = enqueue3(C, kind, C->cap);
        hipError_t ce = hipStreamEndCapture(C->cap, &g);
        if (rc || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return rc ? rc : fail(MPFC_EHIP, std::string("graph capture: ") + hipGetErrorString(ce));
        }
        hipError_t ie = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            gx = nullptr;
            return fail(MPFC_EHIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
        }
    }
    HIP_TRY(hipGraphLaunch(gx, C->stream));
    return MPFC_OK;
}

// Energies of (phi, phiprev, psi) in three dimensions: F (h^3 sums, h times the
// face-difference sum), ||psi||_{-1}^2 = h^3 (psi - mean, w) with -Lap_h w =
// psi - mean (Poisson V-cycles, warm-started by the scheme's recursion for w
// when mu is given), modified energy, mass.
int compute_energies3(mpfc3d_ctx* C, const double* phi, const double* phiprev, const double* psi,
                      const double* mu, double* out) {
    hipStream_t s = C->stream;
    Level3& F0 = C->L[0];
    const size_t total = (size_t)F0.m * F0.n * F0.l;
    const unsigned rb = red_blocks3(total);
    const double ih2 = 1.0 / (F0.h * F0.h);
    const bool warm = C->have_w;
    const bool advance = warm && mu;
    hipLaunchKernelGGL((k_sum2<NT>), dim3(rb), dim3(NT), 0, s, psi, advance ? mu : nullptr, total,
                       C->part, C->pst);
    hipLaunchKernelGGL((k_partials_sum<NT>), dim3(1), dim3(NT), 0, s, C->part, (int)rb, 2, C->acc + 8);
    if (!warm) {
        hipLaunchKernelGGL((k_fill<double>), dim3(blocks256(total)), dim3(256), 0, s, F0.w, total, 0.0);
    } else if (advance) {
        const double sb = C->p.dt * C->p.beta, sM = C->p.dt * C->p.M;
        double a, b;
        if (C->p.scheme == 1) { a = 1.0 / (1.0 + sb); b = sM / (1.0 + sb); }
        else { a = (1.0 - 0.5 * sb) / (1.0 + 0.5 * sb); b = sM / (1.0 + 0.5 * sb); }
        hipLaunchKernelGGL((k_w_advance), dim3(blocks256(total)), dim3(256), 0, s, F0.w, mu, total,
                           a, b, C->acc + 9);
    }
    hipLaunchKernelGGL((k3_p_rhs<NT>), dim3(rb), dim3(NT), 0, s, F0.g, ih2, psi, C->acc + 8, F0.pf,
                       warm ? F0.w : nullptr, C->part);
    hipLaunchKernelGGL((k_partials_sum<NT>), dim3(1), dim3(NT), 0, s, C->part, (int)rb, 2, C->acc + 10);
    if (warm)
        hipLaunchKernelGGL((k_p_finalize<NT>), dim3(1), dim3(NT), 0, s, C->acc + 11, 1, C->pst,
                           C->phist, C->acc + 10, kPoissonRel, kPoissonStall, kPoissonMax);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(C->host_st, C->pst, sizeof(CycleState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int launched = 0;
    while (!C->host_st->done && launched < kPoissonMax) {
        for (int k = 0; k < 2; ++k, ++launched) {
            int rc = run_cycle3(C, 1);
            if (rc) return rc;
        }
        HIP_TRY(hipMemcpyAsync(C->host_st, C->pst, sizeof(CycleState), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    const bool ok = C->host_st->status == ST_CONVERGED;
    C->have_w = true;
    hipLaunchKernelGGL((k3_energy_terms<NT>), dim3(rb), dim3(NT), 0, s, F0.g, ih2, phi, phiprev,
                       F0.pf, F0.w, C->part);
    hipLaunchKernelGGL((k_partials_sum<NT>), dim3(1), dim3(NT), 0, s, C->part, (int)rb, 8, C->acc);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(C->host_buf, C->acc, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double* a = C->host_buf;
    const double h = F0.h, h3 = h * h * h;
    const double Fe = 0.25 * h3 * a[0] + 0.5 * C->alpha * h3 * a[1] - h * a[2] + 0.5 * h3 * a[3];
    out[0] = Fe;
    out[1] = Fe + h3 * a[6] / (2.0 * C->p.M);
    out[2] = out[1] + 0.5 * h * a[5];
    out[3] = h3 * a[4];
    if (!ok) return fail(MPFC_ENOTCONVERGED, "Poisson solve of the -1 norm did not converge");
    return MPFC_OK;
}

}  // namespace

extern "C" {

int mpfc3d_validate(int m, int n, int l, const mpfc_params* p, const mpfc_opts* o) {
    return validate3(m, n, l, p, o);
}

void mpfc3d_destroy(mpfc3d_ctx* C) {
    if (!C) return;
    for (auto& g : C->gx)
        if (g) (void)hipGraphExecDestroy(g);
    if (C->cap) (void)hipStreamDestroy(C->cap);
    for (auto& e : C->ev)
        if (e) (void)hipEventDestroy(e);
    if (C->arena) (void)hipFree(C->arena);
    if (C->host_st) (void)hipHostFree(C->host_st);
    if (C->host_buf) (void)hipHostFree(C->host_buf);
    delete C;
}

int mpfc3d_create(mpfc3d_ctx** out, int m, int n, int l, const mpfc_params* p,
                  const mpfc_opts* o, void* stream) {
    if (!out) return fail(MPFC_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate3(m, n, l, p, o);
    if (rc) return rc;
    mpfc3d_ctx* C = new (std::nothrow) mpfc3d_ctx();
    if (!C) return fail(MPFC_ENOMEM, "host allocation failed");
    C->m = m; C->n = n; C->l = l; C->p = *p; C->o = *o;
    C->stream = (hipStream_t)stream;
    C->alpha = 1.0 - p->eps;
    const double q = p->scheme == 1 ? 1.0 : 2.0;
    C->c = p->dt * p->M / (p->beta + q / p->dt);
    C->d = q / (p->beta + q / p->dt);
    {
        int a = m, b = n, c = l;
        double h = p->h;
        for (;;) {
            Level3 lv;
            lv.m = a; lv.n = b; lv.l = c; lv.h = h; lv.g = make_grid3(a, b, c);
            C->L.push_back(lv);
            int mn = a < b ? a : b;
            mn = mn < c ? mn : c;
            if (mn <= o->coarsest) break;
            a /= 2; b /= 2; c /= 2; h *= 2.0;
        }
    }
    const int nl = (int)C->L.size();
    C->Lp = nl;
    for (int k = 0; k < nl; ++k)
        if ((long long)C->L[k].m * C->L[k].n * C->L[k].l <= CP3_CELLS) { C->Lp = k; break; }
    auto layout = [&](double* base) {
        size_t off = 0;
        auto take = [&](size_t cnt) {
            double* r = base ? base + off : nullptr;
            off += (cnt + 31) & ~(size_t)31;
            return r;
        };
        for (int k = 0; k < nl; ++k) {
            Level3& lv = C->L[k];
            const size_t N = (size_t)lv.m * lv.n * lv.l;
            for (int f = 0; f < 3; ++f) {
                lv.u[f] = take(N);
                lv.f[f] = take(N);
                lv.v[f] = k > 0 ? take(N) : nullptr;
                lv.rr[f] = k > 0 ? take(N) : nullptr;
            }
            lv.xk = p->scheme == 2 ? take(N) : nullptr;
            lv.w = take(N);
            lv.pf = take(N);
            lv.pv = k > 0 ? take(N) : nullptr;
            lv.prr = k > 0 ? take(N) : nullptr;
        }
        C->hist = take(o->max_cycles + 1 + 8);
        C->phist = take(kPoissonMax + 8);
        C->acc = take(64);
        C->nparts = 4096;  // per-block partials (up to 8 values) of at most kRedBlocks3 blocks
        static_assert(kRedBlocks3 <= 4096, "reduction partials exceed the buffer");
        C->part = take((size_t)C->nparts * 8);
        C->st = (CycleState*)take(16);
        C->pst = (CycleState*)take(16);
        return off;
    };
    const size_t bytes = layout(nullptr) * sizeof(double);
    hipError_t e = hipMalloc(&C->arena, bytes);
    if (e != hipSuccess) {
        delete C;
        return fail(MPFC_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    layout((double*)C->arena);
    e = hipHostMalloc((void**)&C->host_st, sizeof(CycleState) * 2, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&C->host_buf, sizeof(double) * (size_t)(o->max_cycles + 64),
                          hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreate(&C->ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&C->ev[1]);
    if (e == hipSuccess) e = hipMemsetAsync(C->arena, 0, bytes, C->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(C->stream);
    if (e != hipSuccess) {
        mpfc3d_destroy(C);
        return fail(MPFC_EHIP, std::string("context setup: ") + hipGetErrorString(e));
    }
    *out = C;
    return MPFC_OK;
}

int mpfc3d_step(mpfc3d_ctx* C, const double* phi_n, const double* phi_nm1, double* psi,
                double* phi_np1, double* mu_out, double* ka_out, mpfc_info* info) {
    if (!C || !phi_n || !psi || !phi_np1) return fail(MPFC_EINVAL, "null argument");
    if (phi_np1 == phi_n || phi_np1 == phi_nm1 || phi_np1 == psi)
        return fail(MPFC_EINVAL, "phi_np1 must not alias the inputs");
    if (!phi_nm1) phi_nm1 = phi_n;
    hipStream_t s = C->stream;
    Level3& F0 = C->L[0];
    const size_t total = (size_t)C->m * C->n * C->l;
    const unsigned nb = blocks256(total);
    const double ih2 = 1.0 / (F0.h * F0.h);
    // source, phi^k on the finest level, guess completed in mu and kappa
    HIP_TRY(hipMemsetAsync(C->st, 0, sizeof(CycleState), s));
    if (C->p.scheme == 1)
        hipLaunchKernelGGL((k3_source<1>), dim3(nb), dim3(256), 0, s, F0.g, ih2, C->d, C->alpha,
                           phi_n, phi_nm1, psi, F0.f[0], F0.f[1], F0.f[2]);
    else
        hipLaunchKernelGGL((k3_source<2>), dim3(nb), dim3(256), 0, s, F0.g, ih2, C->d, C->alpha,
                           phi_n, phi_nm1, psi, F0.f[0], F0.f[1], F0.f[2]);
    hipLaunchKernelGGL(k3_guess, dim3(nb), dim3(256), 0, s, F0.g,
                       C->o.guess == MPFC_GUESS_EXTRAP ? 1 : 0, phi_n, phi_nm1, F0.u[0], F0.xk);
    const LevelOp<double> lo = level_op3(C, F0);
    hipLaunchKernelGGL(k3_complete_kappa, dim3(nb), dim3(256), 0, s, F0.g, ih2, lo.e, F0.u[0],
                       F0.f[2], F0.u[2]);
    if (C->p.scheme == 1)
        hipLaunchKernelGGL((k3_complete_mu<1>), dim3(nb), dim3(256), 0, s, F0.g, ih2, lo.al,
                           F0.u[0], (const double*)nullptr, F0.f[1], F0.u[2], F0.u[1]);
    else
        hipLaunchKernelGGL((k3_complete_mu<2>), dim3(nb), dim3(256), 0, s, F0.g, ih2, lo.al,
                           F0.u[0], F0.xk, F0.f[1], F0.u[2], F0.u[1]);
    // residual of the guess (history entry 0)
    {
        const unsigned rb = red_blocks3(total);
        L3 FF{};
        for (int f = 0; f < 3; ++f) { FF.u[f] = F0.u[f]; FF.f[f] = F0.f[f]; }
        FF.xk = F0.xk;
        const bool nw = C->o.linearization == MPFC_NEWTON;
        if (C->p.scheme == 1) {
            if (nw) hipLaunchKernelGGL((k3_resnorm<MpfcOp3<1, true>, NT>), dim3(rb), dim3(NT), 0, s, MpfcOp3<1, true>{lo}, F0.g, FF, C->part, (const CycleState*)nullptr);
            else hipLaunchKernelGGL((k3_resnorm<MpfcOp3<1, false>, NT>), dim3(rb), dim3(NT), 0, s, MpfcOp3<1, false>{lo}, F0.g, FF, C->part, (const CycleState*)nullptr);
        } else {
            if (nw) hipLaunchKernelGGL((k3_resnorm<MpfcOp3<2, true>, NT>), dim3(rb), dim3(NT), 0, s, MpfcOp3<2, true>{lo}, F0.g, FF, C->part, (const CycleState*)nullptr);
            else hipLaunchKernelGGL((k3_resnorm<MpfcOp3<2, false>, NT>), dim3(rb), dim3(NT), 0, s, MpfcOp3<2, false>{lo}, F0.g, FF, C->part, (const CycleState*)nullptr);
        }
        hipLaunchKernelGGL((k_norm_finalize<NT>), dim3(1), dim3(NT), 0, s, C->part, (int)rb, C->st,
                           C->hist, F0.h * F0.h * F0.h, C->o.tol, C->o.max_cycles + 1,
                           C->o.diverge);
    }
    HIP_TRY(hipGetLastError());
    // cycles: enqueue the expected number, then one or two at a time until the
    // device-side test stops them
    int launched = 0;
    int batch = C->pred > 1 ? C->pred - 1 : 1;
    for (;;) {
        for (int k = 0; k < batch && launched < C->o.max_cycles; ++k, ++launched) {
            int rc = run_cycle3(C, 0);
            if (rc) return rc;
        }
        HIP_TRY(hipMemcpyAsync(C->host_st, C->st, sizeof(CycleState), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (C->host_st->done || launched >= C->o.max_cycles) break;
        batch = 1;
    }
    const CycleState stc = *C->host_st;
    const int cycles = stc.count - 1;
    C->pred = cycles > 0 ? cycles : 1;
    // psi^{k+1} (in place) and phi^{k+1} out; mu and kappa if asked
    if (C->p.scheme == 1)
        hipLaunchKernelGGL((k3_psi_update<1>), dim3(nb), dim3(256), 0, s, F0.g, C->p.dt, F0.u[0],
                           phi_n, psi, phi_np1);
    else
        hipLaunchKernelGGL((k3_psi_update<2>), dim3(nb), dim3(256), 0, s, F0.g, C->p.dt, F0.u[0],
                           phi_n, psi, phi_np1);
    if (mu_out) hipLaunchKernelGGL(k3_from_split, dim3(nb), dim3(256), 0, s, F0.g, F0.u[1], mu_out);
    if (ka_out) hipLaunchKernelGGL(k3_from_split, dim3(nb), dim3(256), 0, s, F0.g, F0.u[2], ka_out);
    HIP_TRY(hipGetLastError());
    double en[4] = {0, 0, 0, 0};
    int erc = MPFC_OK;
    if (C->o.energy) erc = compute_energies3(C, phi_np1, phi_n, psi, F0.u[1], en);
    if (info) {
        info->energy_F = en[0];
        info->energy_pseudo = en[1];
        info->energy_mod = en[2];
        info->mass = en[3];
        info->residual = stc.acc;
        info->n_cycles = cycles;
        info->outer_iters = 0;
        info->energy_status = erc;
        if (info->residual_history && stc.count > 0)
            HIP_TRY(hipMemcpy(info->residual_history, C->hist, sizeof(double) * stc.count,
                              hipMemcpyDeviceToHost));
    }
    HIP_TRY(hipStreamSynchronize(s));
    int rc = status_code(stc.status);
    if (rc == MPFC_OK) rc = erc;
    if (info) info->status = rc;
    if (rc == MPFC_ENOTCONVERGED || rc == MPFC_ENONFINITE || rc == MPFC_EDIVERGED)
        return fail(rc, "three-dimensional step did not converge");
    return rc;
}

int mpfc3d_prof_enable(mpfc3d_ctx* C, int on) {
    if (!C) return fail(MPFC_EINVAL, "ctx is NULL");
    C->prof = on ? 1 : 0;
    return MPFC_OK;
}

int mpfc3d_prof_read(mpfc3d_ctx* C, double* total_ms, long long* launches, long long* cells,
                     int reset) {
    if (!C) return fail(MPFC_EINVAL, "ctx is NULL");
    if (total_ms) *total_ms = C->prof_ms;
    if (launches) *launches = C->prof_launches;
    if (cells) *cells = (long long)C->m * C->n * C->l;
    if (reset) { C->prof_ms = 0; C->prof_launches = 0; }
    return MPFC_OK;
}

}  // extern "C"
