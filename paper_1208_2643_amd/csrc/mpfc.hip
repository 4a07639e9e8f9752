// libmpfc.so: host side of the MPFC nonlinear FAS multigrid time step on one
// gfx950 GPU, behind the C ABI declared in include/mpfc.h.
//
// A step of either convex-splitting scheme (Sec. 3.1, 3.2) solves N(u) = S
// (App. B.1, B.2) by FAS V(nu1, nu2) cycles: red-black nonlinear Gauss-Seidel
// smoothing, residual and 2x2-average restriction, FAS coarse right-hand
// side, dense Newton on the coarsest grid, bilinear prolongation of the
// coarse-grid correction.  The cycle loop is stopped by a device-side test on
// the finest residual norm; the host reads back one small status record per
// cycle.  Afterwards psi is updated (eqs. discrete_1_b / discrete_2_b) and,
// optionally, the energies of Sec. 3 are computed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mpfc.h"
#include "kernels.hpp"
#include "poisson.hpp"

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

Grid make_grid(int m, int n) { return Grid{m, n, ilog2(m), ilog2(n)}; }

constexpr int NT = 256;
const dim3 B2(64, 4);
dim3 grid2(int nx, int ny) { return dim3((nx + 63) / 64, (ny + 3) / 4); }
dim3 grid1(size_t total) { return dim3((unsigned)((total + 255) / 256)); }
unsigned red_blocks(size_t total) {
    size_t b = (total + NT - 1) / NT;
    return (unsigned)(b < 1024 ? b : 1024);
}

struct Level {
    int m = 0, n = 0;
    double h = 0;
    Grid g{};
    double *phi = nullptr, *mu = nullptr, *ka = nullptr;
    double *v0 = nullptr, *v1 = nullptr, *v2 = nullptr;
    double *f0 = nullptr, *f1 = nullptr, *f2 = nullptr;
    double* phik = nullptr;
    double *w = nullptr, *b = nullptr;  // Poisson correction and right-hand side
};

}  // namespace

struct mpfc_ctx {
    int m = 0, n = 0;
    mpfc_params p{};
    mpfc_opts o{};
    hipStream_t stream = nullptr;
    double c = 0, d = 0, alpha = 0;
    std::vector<Level> L;
    double *mu_int = nullptr, *ka_int = nullptr;
    CycleState* st = nullptr;   // nonlinear cycle state
    double* hist = nullptr;     // device residual history
    CycleState* pst = nullptr;  // Poisson cycle state
    double* phist = nullptr;
    double* acc = nullptr;      // reduction accumulators
    double* G = nullptr;        // coarsest Poisson Green's matrix
    int have_w = 0;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    CycleState* host_st = nullptr;  // pinned readback
    double* host_buf = nullptr;     // pinned readback (history / sums)
};

namespace {

LevelOp<double> level_op(const mpfc_ctx* C, const Level& lv) {
    LevelOp<double> op;
    op.ih2 = 1.0 / (lv.h * lv.h);
    op.c = C->c;
    op.al = C->p.scheme == 1 ? C->alpha : 0.5 * C->alpha;
    op.e = C->p.scheme == 1 ? 1.0 : 0.5;
    return op;
}

Fields<double> level_fields(const Level& lv) {
    Fields<double> F;
    F.phi = lv.phi; F.mu = lv.mu; F.ka = lv.ka;
    F.f1 = lv.f0; F.f2 = lv.f1; F.f3 = lv.f2;
    F.phik = lv.phik;
    F.base = nullptr;
    return F;
}

// ---- templated launchers ---------------------------------------------------
template <int S, bool NW>
void launch_smooth(const mpfc_ctx* C, const Level& lv, int sweeps, const CycleState* st,
                   hipStream_t s) {
    const Fields<double> F = level_fields(lv);
    const LevelOp<double> op = level_op(C, lv);
    const dim3 gr = grid2(lv.m / 2, lv.n);
    for (int k = 0; k < sweeps; ++k)
        for (int colour = 0; colour < 2; ++colour)
            hipLaunchKernelGGL((k_smooth_color<double, S, NW, false>), gr, B2, 0, s, F, op, lv.g,
                               colour, st);
}

void smooth(const mpfc_ctx* C, const Level& lv, int sweeps, const CycleState* st, hipStream_t s) {
    const bool nw = C->o.linearization == MPFC_NEWTON;
    if (C->p.scheme == 1) {
        if (nw) launch_smooth<1, true>(C, lv, sweeps, st, s);
        else launch_smooth<1, false>(C, lv, sweeps, st, s);
    } else {
        if (nw) launch_smooth<2, true>(C, lv, sweeps, st, s);
        else launch_smooth<2, false>(C, lv, sweeps, st, s);
    }
}

template <int S>
void launch_restrict_pair(const mpfc_ctx* C, const Level& A, const Level& Bc, const CycleState* st,
                          hipStream_t s) {
    hipLaunchKernelGGL((k_resid_restrict<double, S, false>), grid2(Bc.m, Bc.n), B2, 0, s,
                       level_fields(A), level_op(C, A), A.g, Bc.phi, Bc.mu, Bc.ka, Bc.v0, Bc.v1,
                       Bc.v2, Bc.f0, Bc.f1, Bc.f2, st);
    hipLaunchKernelGGL((k_coarse_rhs<double, S, false>), grid2(Bc.m, Bc.n), B2, 0, s,
                       level_fields(Bc), level_op(C, Bc), Bc.g, Bc.f0, Bc.f1, Bc.f2, st);
}

template <int S>
void launch_coarsest(const mpfc_ctx* C, const Level& lv, const CycleState* st, hipStream_t s) {
    hipLaunchKernelGGL((k_coarsest<double, S, false>), dim3(1), dim3(64), 0, s, level_fields(lv),
                       level_op(C, lv), lv.g, 30, 1e-15, st);
}

void resnorm(mpfc_ctx* C, hipStream_t s) {
    const Level& lv = C->L[0];
    const size_t total = (size_t)lv.m * lv.n;
    const double h2 = lv.h * lv.h;
    const int max_norms = C->o.max_cycles + 1;
    if (C->p.scheme == 1)
        hipLaunchKernelGGL((k_resnorm<1, NT>), dim3(red_blocks(total)), dim3(NT), 0, s,
                           level_fields(lv), level_op(C, lv), lv.g, h2, C->st, C->hist, C->o.tol,
                           max_norms, C->o.diverge, nullptr, nullptr, nullptr);
    else
        hipLaunchKernelGGL((k_resnorm<2, NT>), dim3(red_blocks(total)), dim3(NT), 0, s,
                           level_fields(lv), level_op(C, lv), lv.g, h2, C->st, C->hist, C->o.tol,
                           max_norms, C->o.diverge, nullptr, nullptr, nullptr);
}

// One FAS V(nu1, nu2) cycle on all levels, then the finest residual norm.
void vcycle(mpfc_ctx* C, hipStream_t s) {
    const int nl = (int)C->L.size();
    const CycleState* st = C->st;
    for (int l = 0; l < nl - 1; ++l) {
        smooth(C, C->L[l], C->o.nu1, st, s);
        if (C->p.scheme == 1) launch_restrict_pair<1>(C, C->L[l], C->L[l + 1], st, s);
        else launch_restrict_pair<2>(C, C->L[l], C->L[l + 1], st, s);
    }
    if (C->p.scheme == 1) launch_coarsest<1>(C, C->L[nl - 1], st, s);
    else launch_coarsest<2>(C, C->L[nl - 1], st, s);
    for (int l = nl - 2; l >= 0; --l) {
        const Level& A = C->L[l];
        const Level& Bc = C->L[l + 1];
        hipLaunchKernelGGL((k_prolong_correct<double>), grid2(A.m, A.n), B2, 0, s, A.phi, A.mu,
                           A.ka, A.g, Bc.phi, Bc.mu, Bc.ka, Bc.v0, Bc.v1, Bc.v2, st);
        smooth(C, A, C->o.nu2, st, s);
    }
    resnorm(C, s);
}

// Periodic mean-zero Green's matrix of -Lap_h on an m x n grid of spacing h,
// by the discrete Fourier series: G_pq = (1/(mn)) sum_{k != 0} cos(...)/lambda_k.
void green_matrix(int m, int n, double h, std::vector<double>& G) {
    const int N = m * n;
    G.assign((size_t)N * N, 0.0);
    const double pi = 3.14159265358979323846;
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            const int di = (a % m) - (b % m), dj = (a / m) - (b / m);
            double s = 0.0;
            for (int p = 0; p < m; ++p)
                for (int q = 0; q < n; ++q) {
                    if (p == 0 && q == 0) continue;
                    const double lam = 4.0 / (h * h) *
                                       (std::sin(pi * p / m) * std::sin(pi * p / m) +
                                        std::sin(pi * q / n) * std::sin(pi * q / n));
                    s += std::cos(2.0 * pi * ((double)p * di / m + (double)q * dj / n)) / lam;
                }
            G[(size_t)a * N + b] = s / N;
        }
}

int validate(int m, int n, const mpfc_params* p, const mpfc_opts* o) {
    if (!p) return fail(MPFC_EINVAL, "params is NULL");
    if (!o) return fail(MPFC_EINVAL, "opts is NULL");
    if (!(p->scheme == 1 || p->scheme == 2)) return fail(MPFC_EINVAL, "scheme must be 1 or 2");
    if (!(p->h > 0) || !std::isfinite(p->h)) return fail(MPFC_EINVAL, "h must be > 0");
    if (!(p->dt > 0) || !std::isfinite(p->dt)) return fail(MPFC_EINVAL, "dt must be > 0");
    if (!(p->M > 0) || !std::isfinite(p->M)) return fail(MPFC_EINVAL, "M must be > 0");
    if (!(p->beta >= 0) || !std::isfinite(p->beta)) return fail(MPFC_EINVAL, "beta must be >= 0");
    if (!(p->eps <= 1.0) || !std::isfinite(p->eps)) return fail(MPFC_EINVAL, "eps must be <= 1");
    if (!is_pow2(m) || !is_pow2(n) || m < 2 || n < 2)
        return fail(MPFC_EINVAL, "m and n must be powers of two >= 2");
    if ((long long)m * n > (1LL << 28)) return fail(MPFC_EINVAL, "grid too large (m*n > 2^28)");
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 < 1 || o->nu1 > 8 || o->nu2 > 8)
        return fail(MPFC_EINVAL, "nu1, nu2 must be in [0, 8] with nu1 + nu2 >= 1");
    if (o->max_cycles < 1 || o->max_cycles > 100000)
        return fail(MPFC_EINVAL, "max_cycles must be in [1, 100000]");
    if (!(o->tol > 0)) return fail(MPFC_EINVAL, "tol must be > 0");
    if (!(o->coarsest == 2 || o->coarsest == 4)) return fail(MPFC_EINVAL, "coarsest must be 2 or 4");
    if (!(o->precision == MPFC_FP64 || o->precision == MPFC_MIXED))
        return fail(MPFC_EINVAL, "precision must be MPFC_FP64 or MPFC_MIXED");
    if (!(o->guess == MPFC_GUESS_PREV || o->guess == MPFC_GUESS_EXTRAP))
        return fail(MPFC_EINVAL, "unknown guess mode");
    if (!(o->linearization == MPFC_NEWTON || o->linearization == MPFC_PICARD))
        return fail(MPFC_EINVAL, "unknown linearization");
    if (!(o->diverge > 1.0)) return fail(MPFC_EINVAL, "diverge must be > 1");
    // coarsest grid: coarsen while the smaller side exceeds `coarsest`
    int mm = m, nn = n;
    while ((mm < nn ? mm : nn) > o->coarsest) { mm /= 2; nn /= 2; }
    if (mm * nn > CMAX / 3)
        return fail(MPFC_EINVAL, "aspect ratio too large: coarsest grid exceeds 16 cells");
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

// Energies of (phi, phi_prev, psi) into out[0..3].
int compute_energies(mpfc_ctx* C, const double* phi, const double* phiprev, const double* psi,
                     double* out) {
    hipStream_t s = C->stream;
    const Level& F0 = C->L[0];
    const size_t total = (size_t)C->m * C->n;
    const unsigned rb = red_blocks(total);
    const int nl = (int)C->L.size();
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, C->acc, 16);
    hipLaunchKernelGGL((k_sum<NT>), dim3(rb), dim3(NT), 0, s, psi, total, C->acc + 8);
    hipLaunchKernelGGL((k_p_rhs<NT>), dim3(rb), dim3(NT), 0, s, psi, total, C->acc + 8, F0.b,
                       C->acc + 9);
    if (!C->have_w)
        hipLaunchKernelGGL((k_fill<double>), grid1(total), dim3(256), 0, s, F0.w, total, 0.0);
    hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, C->pst);
    const int pmax = 60;
    const double rtol = 1e-13;
    const double ih2_0 = 1.0 / (F0.h * F0.h);
    hipLaunchKernelGGL((k_p_resnorm<NT>), dim3(rb), dim3(NT), 0, s, F0.w, F0.b, F0.g, ih2_0,
                       C->pst, C->phist, C->acc + 9, rtol, pmax);
    for (int cyc = 0; cyc < pmax; ++cyc) {
        for (int l = 0; l < nl - 1; ++l) {
            const Level& A = C->L[l];
            const Level& Bc = C->L[l + 1];
            for (int sw = 0; sw < 2; ++sw)
                for (int colour = 0; colour < 2; ++colour)
                    hipLaunchKernelGGL(k_p_smooth_color, grid2(A.m / 2, A.n), B2, 0, s, A.w, A.b,
                                       A.g, A.h * A.h, colour, C->pst);
            hipLaunchKernelGGL(k_p_resid_restrict, grid2(Bc.m, Bc.n), B2, 0, s, A.w, A.b, A.g,
                               1.0 / (A.h * A.h), Bc.w, Bc.b, C->pst);
        }
        const Level& Cl = C->L[nl - 1];
        hipLaunchKernelGGL(k_p_coarsest, dim3(1), dim3(64), 0, s, Cl.w, Cl.b, C->G, Cl.m * Cl.n,
                           C->pst);
        for (int l = nl - 2; l >= 0; --l) {
            const Level& A = C->L[l];
            hipLaunchKernelGGL(k_p_prolong, grid2(A.m, A.n), B2, 0, s, A.w, A.g, C->L[l + 1].w,
                               C->pst);
            for (int sw = 0; sw < 2; ++sw)
                for (int colour = 0; colour < 2; ++colour)
                    hipLaunchKernelGGL(k_p_smooth_color, grid2(A.m / 2, A.n), B2, 0, s, A.w, A.b,
                                       A.g, A.h * A.h, colour, C->pst);
        }
        hipLaunchKernelGGL((k_p_resnorm<NT>), dim3(rb), dim3(NT), 0, s, F0.w, F0.b, F0.g, ih2_0,
                           C->pst, C->phist, C->acc + 9, rtol, pmax);
        HIP_TRY(hipMemcpyAsync(C->host_st, C->pst, sizeof(CycleState), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (C->host_st->done) break;
    }
    C->have_w = 1;
    hipLaunchKernelGGL((k_energy_terms<NT>), dim3(rb), dim3(NT), 0, s, F0.g, ih2_0, phi, phiprev,
                       F0.b, F0.w, C->acc);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(C->host_buf, C->acc, 16 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double* a = C->host_buf;
    const double h2 = F0.h * F0.h;
    const double Fe = 0.25 * h2 * a[0] + 0.5 * C->alpha * h2 * a[1] - a[2] + 0.5 * h2 * a[3];
    const double nm1 = h2 * a[6];
    out[0] = Fe;
    out[1] = Fe + nm1 / (2.0 * C->p.M);
    out[2] = out[1] + 0.5 * a[5];
    out[3] = h2 * a[4];
    if (C->host_st->status == ST_NONFINITE)
        return fail(MPFC_ENONFINITE, "non-finite residual in the Poisson solve of the -1 norm");
    return MPFC_OK;
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

int mpfc_create(mpfc_ctx** out, int m, int n, const mpfc_params* p, const mpfc_opts* o,
                void* stream) {
    if (!out) return fail(MPFC_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(m, n, p, o);
    if (rc) return rc;
    if (o->precision != MPFC_FP64)
        return fail(MPFC_EINVAL, "mixed precision is not available in this build");
    mpfc_ctx* C = new (std::nothrow) mpfc_ctx();
    if (!C) return fail(MPFC_ENOMEM, "host allocation failed");
    C->m = m; C->n = n; C->p = *p; C->o = *o;
    C->stream = (hipStream_t)stream;
    C->alpha = 1.0 - p->eps;
    const double q = p->scheme == 1 ? 1.0 : 2.0;
    C->c = p->dt * p->M / (p->beta + q / p->dt);
    C->d = q / (p->beta + q / p->dt);
    // level hierarchy
    {
        int mm = m, nn = n;
        double h = p->h;
        for (;;) {
            Level lv;
            lv.m = mm; lv.n = nn; lv.h = h; lv.g = make_grid(mm, nn);
            C->L.push_back(lv);
            if ((mm < nn ? mm : nn) <= o->coarsest) break;
            mm /= 2; nn /= 2; h *= 2.0;
        }
    }
    const int nl = (int)C->L.size();
    // Arena layout in doubles, every piece 256-byte aligned: the same function
    // sizes the arena (base == nullptr) and then assigns the pointers.
    auto fieldsz = [](const Level& lv) { return (size_t)lv.m * lv.n; };
    const size_t N0 = fieldsz(C->L[0]);
    const Level& Lc = C->L[nl - 1];
    const size_t nG = (size_t)(Lc.m * Lc.n) * (Lc.m * Lc.n);
    auto layout = [&](double* base) {
        size_t off = 0;
        auto take = [&](size_t cnt) {
            double* r = base ? base + off : nullptr;
            off += (cnt + 31) & ~(size_t)31;
            return r;
        };
        Level& F0 = C->L[0];
        F0.f0 = take(N0); F0.f1 = take(N0); F0.f2 = take(N0);
        C->mu_int = take(N0); C->ka_int = take(N0);
        F0.w = take(N0); F0.b = take(N0);
        for (int l = 1; l < nl; ++l) {
            Level& lv = C->L[l];
            const size_t Nl = fieldsz(lv);
            lv.phi = take(Nl); lv.mu = take(Nl); lv.ka = take(Nl);
            lv.v0 = take(Nl); lv.v1 = take(Nl); lv.v2 = take(Nl);
            lv.f0 = take(Nl); lv.f1 = take(Nl); lv.f2 = take(Nl);
            lv.phik = take(Nl);
            lv.w = take(Nl); lv.b = take(Nl);
        }
        C->G = take(nG);
        C->hist = take(o->max_cycles + 1 + 8);
        C->phist = take(o->max_cycles + 1 + 8);
        C->acc = take(64);
        C->st = (CycleState*)take(16);
        C->pst = (CycleState*)take(16);
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
    green_matrix(Lc.m, Lc.n, Lc.h, G);
    e = hipHostMalloc((void**)&C->host_st, sizeof(CycleState) * 2, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&C->host_buf, sizeof(double) * (size_t)(o->max_cycles + 64),
                          hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipMemcpy(C->G, G.data(), nG * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        mpfc_destroy(C);
        return fail(MPFC_EHIP, std::string("context setup: ") + hipGetErrorString(e));
    }
    *out = C;
    return MPFC_OK;
}

void mpfc_destroy(mpfc_ctx* C) {
    if (!C) return;
    if (C->arena) (void)hipFree(C->arena);
    if (C->host_st) (void)hipHostFree(C->host_st);
    if (C->host_buf) (void)hipHostFree(C->host_buf);
    delete C;
}

int mpfc_step(mpfc_ctx* C, const double* phi_n, const double* phi_nm1, double* psi,
              double* phi_np1, double* mu_out, double* ka_out, mpfc_info* info) {
    if (!C) return fail(MPFC_EINVAL, "ctx is NULL");
    if (!phi_n || !psi || !phi_np1) return fail(MPFC_EINVAL, "phi_n, psi and phi_np1 are required");
    if (phi_np1 == phi_n || phi_np1 == phi_nm1 || phi_np1 == psi)
        return fail(MPFC_EINVAL, "phi_np1 must not alias an input");
    if (!phi_nm1) phi_nm1 = phi_n;
    hipStream_t s = C->stream;
    const int nl = (int)C->L.size();
    Level& F0 = C->L[0];
    F0.phi = phi_np1;
    F0.mu = mu_out ? mu_out : C->mu_int;
    F0.ka = ka_out ? ka_out : C->ka_int;
    F0.phik = C->p.scheme == 2 ? const_cast<double*>(phi_n) : nullptr;
    const size_t total = (size_t)C->m * C->n;
    const double ih2 = 1.0 / (F0.h * F0.h);
    // source, phi^k pyramid, guess and its completion
    if (C->p.scheme == 1)
        hipLaunchKernelGGL((k_source<1>), grid2(C->m, C->n), B2, 0, s, F0.g, ih2, C->d, C->alpha,
                           phi_n, phi_nm1, psi, F0.f0, F0.f1, F0.f2);
    else
        hipLaunchKernelGGL((k_source<2>), grid2(C->m, C->n), B2, 0, s, F0.g, ih2, C->d, C->alpha,
                           phi_n, phi_nm1, psi, F0.f0, F0.f1, F0.f2);
    if (C->p.scheme == 2)
        for (int l = 1; l < nl; ++l)
            hipLaunchKernelGGL((k_restrict<double, double>), grid2(C->L[l].m, C->L[l].n), B2, 0, s,
                               C->L[l - 1].g, C->L[l - 1].phik, C->L[l].phik);
    else
        for (int l = 1; l < nl; ++l) C->L[l].phik = nullptr;
    hipLaunchKernelGGL(k_guess, grid1(total), dim3(256), 0, s, F0.g,
                       C->o.guess == MPFC_GUESS_EXTRAP ? 1 : 0, phi_n, phi_nm1, F0.phi);
    const double e = C->p.scheme == 1 ? 1.0 : 0.5;
    const double al = C->p.scheme == 1 ? C->alpha : 0.5 * C->alpha;
    hipLaunchKernelGGL(k_complete_kappa, grid2(C->m, C->n), B2, 0, s, F0.g, ih2, e, F0.phi, F0.f2,
                       F0.ka);
    if (C->p.scheme == 1)
        hipLaunchKernelGGL((k_complete_mu<1>), grid2(C->m, C->n), B2, 0, s, F0.g, ih2, al, F0.phi,
                           F0.phik, F0.ka, F0.f1, F0.mu);
    else
        hipLaunchKernelGGL((k_complete_mu<2>), grid2(C->m, C->n), B2, 0, s, F0.g, ih2, al, F0.phi,
                           F0.phik, F0.ka, F0.f1, F0.mu);
    hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, C->st);
    resnorm(C, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(C->host_st, C->st, sizeof(CycleState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int guard = 0; !C->host_st->done; ++guard) {
        if (guard > C->o.max_cycles + 1)
            return fail(MPFC_EHIP, "internal: cycle state did not advance");
        vcycle(C, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(C->host_st, C->st, sizeof(CycleState), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    const CycleState fin = *C->host_st;
    const int ncyc = fin.count - 1;
    // psi update
    if (C->p.scheme == 1)
        hipLaunchKernelGGL((k_psi_update<1>), grid1(total), dim3(256), 0, s, total, C->p.dt, F0.phi,
                           phi_n, psi);
    else
        hipLaunchKernelGGL((k_psi_update<2>), grid1(total), dim3(256), 0, s, total, C->p.dt, F0.phi,
                           phi_n, psi);
    HIP_TRY(hipGetLastError());
    const int rc = status_code(fin.status);
    double en[4] = {0, 0, 0, 0};
    if (C->o.energy) {
        const int erc = compute_energies(C, F0.phi, phi_n, psi, en);
        if (erc && erc != MPFC_ENONFINITE) return erc;
    }
    if (info) {
        info->n_cycles = ncyc;
        info->status = rc;
        info->outer_iters = 0;
        info->energy_F = en[0];
        info->energy_pseudo = en[1];
        info->energy_mod = en[2];
        info->mass = en[3];
        HIP_TRY(hipMemcpyAsync(C->host_buf, C->hist, sizeof(double) * fin.count,
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        info->residual = C->host_buf[fin.count - 1];
        if (info->residual_history)
            std::memcpy(info->residual_history, C->host_buf, sizeof(double) * fin.count);
    } else {
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (rc) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "step stopped with status %d after %d cycles", fin.status,
                      ncyc);
        return fail(rc, buf);
    }
    return MPFC_OK;
}

int mpfc_energies(mpfc_ctx* C, const double* phi, const double* phi_prev, const double* psi,
                  double* out) {
    if (!C || !phi || !psi || !out) return fail(MPFC_EINVAL, "ctx, phi, psi and out are required");
    return compute_energies(C, phi, phi_prev, psi, out);
}

// ---- operator-level entry points --------------------------------------------
int mpfc_op_smooth(int scheme, int linearization, int m, int n, double h, double c, double alpha,
                   const double* phik, double* phi, double* mu, double* ka, const double* f1,
                   const double* f2, const double* f3, int sweeps, void* stream) {
    if (!(scheme == 1 || scheme == 2) || !is_pow2(m) || !is_pow2(n) || m < 2 || n < 2 ||
        sweeps < 0 || !(h > 0) || !phi || !mu || !ka || !f1 || !f2 || !f3 ||
        (scheme == 2 && !phik))
        return fail(MPFC_EINVAL, "mpfc_op_smooth: bad arguments");
    mpfc_ctx C;
    C.p.scheme = scheme;
    C.c = c; C.alpha = alpha;
    C.o.linearization = linearization;
    Level lv;
    lv.m = m; lv.n = n; lv.h = h; lv.g = make_grid(m, n);
    lv.phi = phi; lv.mu = mu; lv.ka = ka;
    lv.f0 = const_cast<double*>(f1); lv.f1 = const_cast<double*>(f2); lv.f2 = const_cast<double*>(f3);
    lv.phik = const_cast<double*>(phik);
    smooth(&C, lv, sweeps, nullptr, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return MPFC_OK;
}

int mpfc_op_residual(int scheme, int m, int n, double h, double c, double alpha,
                     const double* phik, const double* phi, const double* mu, const double* ka,
                     const double* f1, const double* f2, const double* f3, double* r1, double* r2,
                     double* r3, void* stream) {
    if (!(scheme == 1 || scheme == 2) || !is_pow2(m) || !is_pow2(n) || m < 2 || n < 2 ||
        !(h > 0) || !phi || !mu || !ka || !f1 || !f2 || !f3 || !r1 || !r2 || !r3 ||
        (scheme == 2 && !phik))
        return fail(MPFC_EINVAL, "mpfc_op_residual: bad arguments");
    Fields<double> F;
    F.phi = const_cast<double*>(phi); F.mu = const_cast<double*>(mu); F.ka = const_cast<double*>(ka);
    F.f1 = f1; F.f2 = f2; F.f3 = f3; F.phik = phik; F.base = nullptr;
    LevelOp<double> op;
    op.ih2 = 1.0 / (h * h); op.c = c;
    op.al = scheme == 1 ? alpha : 0.5 * alpha;
    op.e = scheme == 1 ? 1.0 : 0.5;
    const Grid g = make_grid(m, n);
    hipStream_t s = (hipStream_t)stream;
    if (scheme == 1)
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
    if (!p || !(p->scheme == 1 || p->scheme == 2) || !is_pow2(m) || !is_pow2(n) || m < 2 ||
        n < 2 || !(p->h > 0) || !(p->dt > 0) || !phik || !psik || !S1 || !S2 || !S3)
        return fail(MPFC_EINVAL, "mpfc_op_source: bad arguments");
    if (!phikm1) phikm1 = phik;
    const double q = p->scheme == 1 ? 1.0 : 2.0;
    const double d = q / (p->beta + q / p->dt);
    const Grid g = make_grid(m, n);
    hipStream_t s = (hipStream_t)stream;
    if (p->scheme == 1)
        hipLaunchKernelGGL((k_source<1>), grid2(m, n), B2, 0, s, g, 1.0 / (p->h * p->h), d,
                           1.0 - p->eps, phik, phikm1, psik, S1, S2, S3);
    else
        hipLaunchKernelGGL((k_source<2>), grid2(m, n), B2, 0, s, g, 1.0 / (p->h * p->h), d,
                           1.0 - p->eps, phik, phikm1, psik, S1, S2, S3);
    HIP_TRY(hipGetLastError());
    return MPFC_OK;
}

int mpfc_op_restrict(int m, int n, const double* fine, double* coarse, void* stream) {
    if (!is_pow2(m) || !is_pow2(n) || m < 2 || n < 2 || !fine || !coarse)
        return fail(MPFC_EINVAL, "mpfc_op_restrict: bad arguments");
    hipLaunchKernelGGL((k_restrict<double, double>), grid2(m / 2, n / 2), B2, 0,
                       (hipStream_t)stream, make_grid(m, n), fine, coarse);
    HIP_TRY(hipGetLastError());
    return MPFC_OK;
}

int mpfc_op_prolong_correct(int m, int n, const double* uH0, const double* uH1,
                            const double* uH2, const double* vH0, const double* vH1,
                            const double* vH2, double* u0, double* u1, double* u2, void* stream) {
    if (!is_pow2(m) || !is_pow2(n) || m < 4 || n < 4 || !uH0 || !uH1 || !uH2 || !vH0 || !vH1 ||
        !vH2 || !u0 || !u1 || !u2)
        return fail(MPFC_EINVAL, "mpfc_op_prolong_correct: bad arguments");
    hipLaunchKernelGGL((k_prolong_correct<double>), grid2(m, n), B2, 0, (hipStream_t)stream, u0,
                       u1, u2, make_grid(m, n), uH0, uH1, uH2, vH0, vH1, vH2, nullptr);
    HIP_TRY(hipGetLastError());
    return MPFC_OK;
}

}  // extern "C"
