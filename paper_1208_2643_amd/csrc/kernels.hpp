// Device kernels of the MPFC nonlinear FAS multigrid time step, for gfx950.
//
// One implicit step of either convex-splitting scheme (first order: Sec. 3.1,
// second order: Sec. 3.2) is the solve of N(u) = S for u = (phi, mu, kappa)
// on a cell-centred grid (App. B.1 / B.2), followed by the psi update (eqs.
// discrete_1_b / discrete_2_b).  Storage: every field is an m x n array,
// row-major with x fastest (index j*m + i); ghost cells (App. A) are index
// maps per axis: periodic wrap-around (m and n are powers of two, so a bit
// mask) or, on a homogeneous Neumann axis, the reflection about the boundary.
//
// Kernels are templated on the arithmetic type T (double, or float for the
// inner cycles of mixed precision) and on the scheme.  DEFECT = true selects
// the correction equation used by mixed precision: the unknown is a
// correction e to a base state u_b held as a coefficient field, and the
// nonlinear term is g(phi_b + e) - g(phi_b) written in factored form, so no
// cancellation happens in low precision.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpfc {

// Stop/bookkeeping state of the cycle loop, kept on the device so that the
// loop can run without a host round trip per kernel.
struct CycleState {
    double acc;          // latest residual norm (written with hist[count - 1])
    unsigned int blocks; // blocks that have added to acc
    int count;           // norms recorded so far (entries of hist)
    int status;          // 0 running, 1 converged, 2 cycle limit, 3 non-finite, 4 diverged
    int done;            // status != 0; every cycle kernel returns at once when set
    int pad0, pad1;
};

enum { ST_RUNNING = 0, ST_CONVERGED = 1, ST_MAXCYC = 2, ST_NONFINITE = 3, ST_DIVERGED = 4 };

__device__ __forceinline__ bool stopped(const CycleState* st) {
    return st != nullptr && st->done != 0;
}

// ---------------------------------------------------------------------------
// Nonlinear term of N^(2) (App. B.1: phi^3; App. B.2: chi(phi, phi^k)(phi + phi^k)/2
// with chi(a, b) = (a^2 + b^2)/2) and its derivative.  In DEFECT mode v is a
// correction to the base value pb and the value is g(pb + v) - g(pb).
template <typename T, int SCHEME, bool DEFECT>
__device__ __forceinline__ T nl_value(T v, T pb, T xk) {
    if constexpr (!DEFECT) {
        if constexpr (SCHEME == 1) return v * v * v;
        else return T(0.25) * (v * v + xk * xk) * (v + xk);
    } else {
        if constexpr (SCHEME == 1) {
            // (pb+v)^3 - pb^3 = v (3 pb^2 + 3 pb v + v^2)
            return v * (T(3) * pb * pb + T(3) * pb * v + v * v);
        } else {
            // [((pb+v)^2 + xk^2)(pb+v+xk) - (pb^2 + xk^2)(pb+xk)]/4
            //   = v [3 pb^2 + 2 pb xk + xk^2 + v (3 pb + xk) + v^2]/4
            return T(0.25) * v *
                   (T(3) * pb * pb + T(2) * pb * xk + xk * xk + v * (T(3) * pb + xk) + v * v);
        }
    }
}

// d/dv of the nonlinear term (Newton) or the Picard coefficient, both taken
// at the full value x = pb + v.
template <typename T, int SCHEME, bool NEWTON>
__device__ __forceinline__ T nl_lin(T x, T xk) {
    if constexpr (SCHEME == 1) {
        return NEWTON ? T(3) * x * x : x * x;
    } else {
        if constexpr (NEWTON) return T(0.25) * (T(3) * x * x + T(2) * x * xk + xk * xk);
        else return T(0.25) * (x * x + xk * xk);  // chi(x, xk)/2
    }
}

// Per-level operator constants.
template <typename T>
struct LevelOp {
    T ih2;   // 1/h^2
    T c;     // s M/(beta + 1/s) or s M/(beta + 2/s)
    T al;    // alpha (scheme 1) or alpha/2 (scheme 2)
    T e;     // 1 (scheme 1) or 1/2 (scheme 2): N^(3) = kappa - e Lap phi
};

// Boundary conditions, per axis (App. A): periodic (eqs. per-bcs) unless the
// axis' bit is set, then homogeneous Neumann (eqs. h-n-bcs).
constexpr int BC_NEUMANN_X = 1, BC_NEUMANN_Y = 2;

struct Grid {
    int m, n;       // cells along x and y
    int lm, ln;     // log2 m, log2 n; -1 for a side that is not a power of two
    int bc;         // BC_NEUMANN_X | BC_NEUMANN_Y bits
};

// Cell holding the value of (ghost or interior) cell i along an axis of m
// cells.  Periodic: wrap-around.  Neumann: the even reflection about the
// boundary edges (period 2m), so the first ghost repeats the boundary cell
// and deeper ghosts (tile halos) mirror the interior.  axis_index needs m a
// power of two; axis_index_any takes any m.
__device__ __forceinline__ int axis_index(int i, int m, bool neumann) {
    if (!neumann) return i & (m - 1);
    const int r = i & (2 * m - 1);
    return r < m ? r : 2 * m - 1 - r;
}
__device__ __forceinline__ int axis_index_any(int i, int m, bool neumann) {
    if (!neumann) {
        const int r = i % m;
        return r < 0 ? r + m : r;
    }
    int r = i % (2 * m);
    if (r < 0) r += 2 * m;
    return r < m ? r : 2 * m - 1 - r;
}
// One step outside the axis (i in [-m, 2m)), any m: compares and selects, no
// branch and no division; the per-cell kernels only look one cell across.
__device__ __forceinline__ int wrap1(int i, int m, bool neumann) {
    const int lo = neumann ? -1 - i : i + m;
    const int hi = neumann ? 2 * m - 1 - i : i - m;
    return i < 0 ? lo : (i >= m ? hi : i);
}
__device__ __forceinline__ int wrapx(int i, const Grid& g) {
    return wrap1(i, g.m, g.bc & BC_NEUMANN_X);
}
__device__ __forceinline__ int wrapy(int j, const Grid& g) {
    return wrap1(j, g.n, g.bc & BC_NEUMANN_Y);
}
__device__ __forceinline__ size_t at(int i, int j, const Grid& g) {
    const unsigned r = g.lm >= 0 ? (unsigned)j << g.lm : (unsigned)j * (unsigned)g.m;
    return (size_t)r + (size_t)i;   // m * n <= 2^28
}
// (i, j) of the cell at linear index q (< 2^28).
__device__ __forceinline__ void cell_of(size_t q, const Grid& g, int& i, int& j) {
    const unsigned u = (unsigned)q;
    if (g.lm >= 0) {
        i = (int)(u & (unsigned)(g.m - 1));
        j = (int)(u >> g.lm);
    } else {
        j = (int)(u / (unsigned)g.m);
        i = (int)(u - (unsigned)j * (unsigned)g.m);
    }
}

// Sum of the four neighbours of (i, j).
template <typename T>
__device__ __forceinline__ T nsum(const T* __restrict__ f, int i, int j, const Grid& g) {
    const int ip = wrapx(i + 1, g), im = wrapx(i - 1, g);
    const int jp = wrapy(j + 1, g), jm = wrapy(j - 1, g);
    return (f[at(ip, j, g)] + f[at(im, j, g)]) + (f[at(i, jp, g)] + f[at(i, jm, g)]);
}

// Fields of one level.
template <typename T>
struct Fields {
    T* phi; T* mu; T* ka;          // unknown u (in DEFECT mode: the correction)
    const T* f1; const T* f2; const T* f3;  // right-hand side (S, or FAS coarse RHS)
    const T* phik;                 // phi^k on this level (scheme 2), else null
    const T* base;                 // base phi (DEFECT mode), else null
    const T* pin = nullptr;        // pinning weight W on this level (Sec. 4.4), else null
};

// r = f - N(u) at one cell.
template <typename T, int SCHEME, bool DEFECT>
__device__ __forceinline__ void residual_at(const Fields<T>& F, const LevelOp<T>& op,
                                            const Grid& g, int i, int j, T& r1, T& r2, T& r3) {
    const size_t q = at(i, j, g);
    const T x = F.phi[q], y = F.mu[q], z = F.ka[q];
    const T xk = (SCHEME == 2) ? F.phik[q] : T(0);
    const T pb = DEFECT ? F.base[q] : T(0);
    const T lphi = (nsum(F.phi, i, j, g) - T(4) * x) * op.ih2;
    const T lmu = (nsum(F.mu, i, j, g) - T(4) * y) * op.ih2;
    const T lka = (nsum(F.ka, i, j, g) - T(4) * z) * op.ih2;
    const T al = op.al + (F.pin ? F.pin[q] : T(0));  // pinning adds W to the phi coefficient
    r1 = F.f1[q] - (x - op.c * lmu);
    r2 = F.f2[q] - (y - nl_value<T, SCHEME, DEFECT>(x, pb, xk) - al * x - lka);
    r3 = F.f3[q] - (z - op.e * lphi);
}

// Nonlinear collective Gauss-Seidel update of one cell (App. B): the 3x3
// system J_loc * delta = r, J_loc = [[1, a, 0], [-d, 1, b], [ec, 0, 1]],
// a = 4c/h^2, b = 4/h^2, ec = 4e/h^2, d = al + linearised nonlinear
// coefficient, solved by elimination (equivalent to Cramer's rule; one
// division).
template <typename T, int SCHEME, bool NEWTON, bool DEFECT>
__device__ __forceinline__ void relax_at(const Fields<T>& F, const LevelOp<T>& op, const Grid& g,
                                         int i, int j) {
    T r1, r2, r3;
    residual_at<T, SCHEME, DEFECT>(F, op, g, i, j, r1, r2, r3);
    const size_t q = at(i, j, g);
    const T x = F.phi[q];
    const T xk = (SCHEME == 2) ? F.phik[q] : T(0);
    const T pb = DEFECT ? F.base[q] : T(0);
    const T d = op.al + (F.pin ? F.pin[q] : T(0)) + nl_lin<T, SCHEME, NEWTON>(pb + x, xk);
    const T a = T(4) * op.c * op.ih2, b = T(4) * op.ih2, ec = T(4) * op.e * op.ih2;
    const T det = T(1) + a * d + a * b * ec;
    const T dm = (r2 + (d + b * ec) * r1 - b * r3) / det;
    const T dx = r1 - a * dm;
    const T dk = r3 - ec * dx;
    F.phi[q] = x + dx;
    F.mu[q] += dm;
    F.ka[q] += dk;
}

// r = f - N(u) on every cell (operator-level entry point).
template <typename T, int SCHEME, bool DEFECT>
__global__ void __launch_bounds__(256) k_residual_field(Fields<T> F, LevelOp<T> op, Grid g, T* r0,
                                                        T* r1, T* r2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.m || j >= g.n) return;
    T a, b, c;
    residual_at<T, SCHEME, DEFECT>(F, op, g, i, j, a, b, c);
    const size_t q = at(i, j, g);
    r0[q] = a; r1[q] = b; r2[q] = c;
}

// ---------------------------------------------------------------------------
// Block-wide sum of doubles: wave shuffles, then one value per wave in LDS.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) t += red[w];
    }
    return t;  // valid in thread 0
}

// Stop test after a norm: every block of the producing kernel wrote the sum
// of its squares to part[b]; one block adds them in a fixed order, records
// ||r|| = sqrt(h2 * sum) in hist[count] and sets the status: converged when
// ||r|| <= tol, non-finite, diverged (growth by `diverge` over hist[0]) or the
// cycle limit.  No atomics and no device-wide fences are involved, and the
// norm is deterministic.
template <int NT>
__device__ __forceinline__ void norm_finalize_body(const double* __restrict__ part, int nparts,
                                                   CycleState* st, double* hist, double h2,
                                                   double tol, int max_norms, double diverge) {
    __shared__ double red[NT / 64];
    double s = 0.0;
    for (int b = threadIdx.x; b < nparts; b += NT) s += part[b];
    const double tot = block_sum<NT>(s, red);
    if (threadIdx.x == 0) {
        const double nr = sqrt(h2 * tot);
        const int k = st->count;
        hist[k] = nr;
        st->acc = nr;  // latest norm, read back with the state
        st->count = k + 1;
        int status = ST_RUNNING;
        if (!(nr == nr) || nr > 1.0e300) status = ST_NONFINITE;
        else if (nr <= tol) status = ST_CONVERGED;
        else if (k > 0 && nr > diverge * hist[0]) status = ST_DIVERGED;
        else if (k + 1 >= max_norms) status = ST_MAXCYC;
        st->status = status;
        st->done = status != ST_RUNNING;
    }
}

template <int NT>
__global__ void __launch_bounds__(NT) k_norm_finalize(const double* __restrict__ part, int nparts,
                                                      CycleState* st, double* hist, double h2,
                                                      double tol, int max_norms, double diverge) {
    if (stopped(st)) return;
    norm_finalize_body<NT>(part, nparts, st, hist, h2, tol, max_norms, diverge);
}

// Finest-grid residual sum of squares sum_c sum_ij r_c^2 (FP64, the stopping
// test; k_norm_finalize turns the per-block sums into the norm).  With r0
// non-null the residual is also stored.
template <int SCHEME, int NT>
__global__ void __launch_bounds__(NT) k_resnorm(Fields<double> F, LevelOp<double> op, Grid g,
                                                const CycleState* st, double* part, double* r0,
                                                double* r1o, double* r2o) {
    if (stopped(st)) return;
    __shared__ double red[NT / 64];
    double acc = 0.0;
    const size_t total = (size_t)g.m * g.n;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        int i, j;
        cell_of(q, g, i, j);
        double a, b, c;
        residual_at<double, SCHEME, false>(F, op, g, i, j, a, b, c);
        acc += a * a + b * b + c * c;
        if (r0) { r0[q] = a; r1o[q] = b; r2o[q] = c; }
    }
    const double bs = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;  // summed by k_norm_finalize
}

// Mixed precision, outer FP64 defect-correction step on the finest grid, one
// cell: u_new = u + e (the FP32 correction; `add` = 0 keeps u, for the first
// residual of a step), r = S - N(u_new) in FP64, and the inputs of the next
// FP32 correction solve: r rounded to FP32 and the base phi rounded to FP32.
// The neighbours' u + e are recomputed here, so no other thread's write is
// read.  Returns the cell's sum of squared residuals (the stopping test).
template <int SCHEME>
__device__ __forceinline__ double defect_cell(const Fields<double>& F, const LevelOp<double>& op,
                                              const Grid& g, const float* __restrict__ e0,
                                              const float* __restrict__ e1,
                                              const float* __restrict__ e2, int add, double* un0,
                                              double* un1, double* un2, float* r0, float* r1,
                                              float* r2, float* pbase, int i, int j) {
    const size_t q = at(i, j, g);
    const size_t nb[4] = {at(wrapx(i + 1, g), j, g), at(wrapx(i - 1, g), j, g),
                          at(i, wrapy(j + 1, g), g), at(i, wrapy(j - 1, g), g)};
    auto val = [&](const double* u, const float* e, size_t k) {
        return add ? u[k] + (double)e[k] : u[k];
    };
    const double x = val(F.phi, e0, q), y = val(F.mu, e1, q), z = val(F.ka, e2, q);
    double sx = 0, sy = 0, sz = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        sx += val(F.phi, e0, nb[k]);
        sy += val(F.mu, e1, nb[k]);
        sz += val(F.ka, e2, nb[k]);
    }
    const double xk = SCHEME == 2 ? F.phik[q] : 0.0;
    const double lphi = (sx - 4.0 * x) * op.ih2;
    const double lmu = (sy - 4.0 * y) * op.ih2;
    const double lka = (sz - 4.0 * z) * op.ih2;
    const double a = F.f1[q] - (x - op.c * lmu);
    const double b = F.f2[q] - (y - nl_value<double, SCHEME, false>(x, 0.0, xk) - op.al * x - lka);
    const double c = F.f3[q] - (z - op.e * lphi);
    un0[q] = x; un1[q] = y; un2[q] = z;
    r0[q] = (float)a; r1[q] = (float)b; r2[q] = (float)c;
    pbase[q] = (float)x;
    return a * a + b * b + c * c;
}

// Whole finest grid, one thread per cell; per-block sums of r^2 into part[]
// (summed by k_norm_finalize).  The correction e is cleared by the next
// outer iteration, not here (neighbours still read it).
template <int SCHEME, int NT>
__global__ void __launch_bounds__(NT) k_defect(Fields<double> F, LevelOp<double> op, Grid g,
                                               const CycleState* st, double* part,
                                               const float* __restrict__ e0,
                                               const float* __restrict__ e1,
                                               const float* __restrict__ e2, int add,
                                               double* un0, double* un1, double* un2,
                                               float* r0, float* r1, float* r2, float* pbase) {
    if (stopped(st)) return;
    __shared__ double red[NT / 64];
    double acc = 0.0;
    const size_t total = (size_t)g.m * g.n;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        int i, j;
        cell_of(q, g, i, j);
        acc += defect_cell<SCHEME>(F, op, g, e0, e1, e2, add, un0, un1, un2, r0, r1, r2, pbase, i, j);
    }
    const double bs = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(256) k_convert(const TI* __restrict__ a, TO* b, size_t n) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) b[q] = (TO)a[q];
}

__global__ void k_state_reset(CycleState* st) {
    if (threadIdx.x == 0) {
        st->acc = 0.0; st->blocks = 0u; st->count = 0;
        st->status = ST_RUNNING; st->done = 0; st->pad0 = st->pad1 = 0;
    }
}

// ---------------------------------------------------------------------------
// Step set-up and wrap-up kernels (one thread per cell).

// Source S (App. B.1 / B.2) at cell (i, j).  d = weight of psi^k.  With the
// pinning of Sec. 4.4 (scheme 2; pin != null) S^(2) gains W (phi^k - 2 phi_hat):
// the unknown mu is then mu~ = mu + 2 ((phi^{k+1} + phi^k)/2 - phi_hat) W.
template <int SCHEME>
__device__ __forceinline__ void source_cell(const Grid& g, double ih2, double d, double alpha,
                                            const double* __restrict__ phik,
                                            const double* __restrict__ phikm1,
                                            const double* __restrict__ psik, double* S1,
                                            double* S2, double* S3, double* phik_copy, int i,
                                            int j, const double* __restrict__ pin = nullptr,
                                            const double* __restrict__ phihat = nullptr) {
    const size_t q = at(i, j, g);
    const double pk = phik[q];
    if (phik_copy) phik_copy[q] = pk;
    const double lk = (nsum(phik, i, j, g) - 4.0 * pk) * ih2;
    S1[q] = pk + d * psik[q];
    if constexpr (SCHEME == 1) {
        S2[q] = 2.0 * lk;
        S3[q] = 0.0;
    } else {
        // 2 Lap((3 phi^k - phi^{k-1})/2) = 3 Lap phi^k - Lap phi^{k-1}
        const double lkm1 = (nsum(phikm1, i, j, g) - 4.0 * phikm1[q]) * ih2;
        S2[q] = 0.5 * alpha * pk + (3.0 * lk - lkm1);
        if (pin) S2[q] += pin[q] * (pk - 2.0 * phihat[q]);
        S3[q] = 0.5 * lk;
    }
}

template <int SCHEME>
__global__ void __launch_bounds__(256) k_source(Grid g, double ih2, double d, double alpha,
                                                const double* __restrict__ phik,
                                                const double* __restrict__ phikm1,
                                                const double* __restrict__ psik, double* S1,
                                                double* S2, double* S3, double* phik_copy,
                                                const double* __restrict__ pin,
                                                const double* __restrict__ phihat) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.m || j >= g.n) return;
    source_cell<SCHEME>(g, ih2, d, alpha, phik, phikm1, psik, S1, S2, S3, phik_copy, i, j, pin,
                        phihat);
}

// Initial guess phi^(0): phi^k (mode 0) or 2 phi^k - phi^{k-1} (mode 1).
__device__ __forceinline__ double guess_value(int mode, double pk, double pkm1) {
    return mode == 1 ? 2.0 * pk - pkm1 : pk;
}

__global__ void __launch_bounds__(256) k_guess(Grid g, int mode, const double* __restrict__ phik,
                                               const double* __restrict__ phikm1, double* phi) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (size_t)g.m * g.n) return;
    phi[q] = guess_value(mode, phik[q], phikm1[q]);
}

// Consistent completion of the guess: kappa = S3 + e Lap phi (so N^(3) = S^(3)).
__device__ __forceinline__ void complete_kappa_cell(const Grid& g, double ih2, double e,
                                                    const double* __restrict__ phi,
                                                    const double* __restrict__ S3, double* ka,
                                                    int i, int j) {
    const size_t q = at(i, j, g);
    ka[q] = S3[q] + e * (nsum(phi, i, j, g) - 4.0 * phi[q]) * ih2;
}

// Step set-up in one pass (extrapolated or previous-step guess): the source S
// (source_cell), the guess phi0 = guess_value(mode, phi^k, phi^{k-1}) and
// kappa = S3 + e Lap phi0, the first half of the guess's completion.  Each
// thread forms the guess at its four neighbours itself, so no other thread's
// output is read; the arithmetic is that of k_guess and complete_kappa_cell.
// Workgroup (0, 0) also resets the cycle state.
template <int SCHEME>
__global__ void __launch_bounds__(256) k_setup(Grid g, double ih2, double d, double alpha,
                                               double e, int mode,
                                               const double* __restrict__ phik,
                                               const double* __restrict__ phikm1,
                                               const double* __restrict__ psik, double* S1,
                                               double* S2, double* S3, double* phik_copy,
                                               const double* __restrict__ pin,
                                               const double* __restrict__ phihat, double* phi0,
                                               double* ka, CycleState* st) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && threadIdx.y == 0) {
        st->acc = 0.0; st->blocks = 0u; st->count = 0;
        st->status = ST_RUNNING; st->done = 0; st->pad0 = st->pad1 = 0;
    }
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.m || j >= g.n) return;
    source_cell<SCHEME>(g, ih2, d, alpha, phik, phikm1, psik, S1, S2, S3, phik_copy, i, j, pin,
                        phihat);
    const size_t q = at(i, j, g);
    auto gv = [&](size_t k) { return guess_value(mode, phik[k], phikm1[k]); };
    const double x = gv(q);
    phi0[q] = x;
    const int ip = wrapx(i + 1, g), im = wrapx(i - 1, g);
    const int jp = wrapy(j + 1, g), jm = wrapy(j - 1, g);
    const double ns = (gv(at(ip, j, g)) + gv(at(im, j, g))) + (gv(at(i, jp, g)) + gv(at(i, jm, g)));
    ka[q] = S3[q] + e * (ns - 4.0 * x) * ih2;
}

// Residual norm of a guess completed by k_setup and k_complete_mu: N^(2) = S^(2)
// and N^(3) = S^(3) hold by construction (up to rounding), so only
// r1 = S1 - (phi - c Lap mu) is summed (per-block sums of r1^2 into part[];
// k_norm_finalize turns them into the norm).  Reads phi, mu and S1.
template <int NT>
__global__ void __launch_bounds__(NT) k_resnorm_guess(Fields<double> F, LevelOp<double> op, Grid g,
                                                      double* part) {
    __shared__ double red[NT / 64];
    double acc = 0.0;
    const size_t total = (size_t)g.m * g.n;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        int i, j;
        cell_of(q, g, i, j);
        const double lmu = (nsum(F.mu, i, j, g) - 4.0 * F.mu[q]) * op.ih2;
        const double r1 = F.f1[q] - (F.phi[q] - op.c * lmu);
        acc += r1 * r1;
    }
    const double bs = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

__global__ void __launch_bounds__(256) k_complete_kappa(Grid g, double ih2, double e,
                                                        const double* __restrict__ phi,
                                                        const double* __restrict__ S3,
                                                        double* ka) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.m || j >= g.n) return;
    complete_kappa_cell(g, ih2, e, phi, S3, ka, i, j);
}

// ... and mu = S2 + g(phi) + al phi + Lap kappa (so N^(2) = S^(2)).
template <int SCHEME>
__device__ __forceinline__ void complete_mu_cell(const Grid& g, double ih2, double al,
                                                 const double* __restrict__ phi,
                                                 const double* __restrict__ phik,
                                                 const double* __restrict__ ka,
                                                 const double* __restrict__ S2, double* mu, int i,
                                                 int j, const double* __restrict__ pin = nullptr) {
    const size_t q = at(i, j, g);
    const double x = phi[q];
    const double xk = SCHEME == 2 ? phik[q] : 0.0;
    const double alq = al + (pin ? pin[q] : 0.0);
    mu[q] = S2[q] + nl_value<double, SCHEME, false>(x, 0.0, xk) + alq * x +
            (nsum(ka, i, j, g) - 4.0 * ka[q]) * ih2;
}

template <int SCHEME>
__global__ void __launch_bounds__(256) k_complete_mu(Grid g, double ih2, double al,
                                                     const double* __restrict__ phi,
                                                     const double* __restrict__ phik,
                                                     const double* __restrict__ ka,
                                                     const double* __restrict__ S2, double* mu,
                                                     const double* __restrict__ pin) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.m || j >= g.n) return;
    complete_mu_cell<SCHEME>(g, ih2, al, phi, phik, ka, S2, mu, i, j, pin);
}

// 2x2 average (restriction of phi^k for the scheme-2 coarse operators).
template <typename TI, typename TO>
__global__ void __launch_bounds__(256) k_restrict(Grid g, const TI* __restrict__ f, TO* fc) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int mc = g.m >> 1, nc = g.n >> 1;
    if (I >= mc || J >= nc) return;
    const TI s = (f[at(2 * I, 2 * J, g)] + f[at(2 * I + 1, 2 * J, g)]) +
                 (f[at(2 * I, 2 * J + 1, g)] + f[at(2 * I + 1, 2 * J + 1, g)]);
    fc[(size_t)J * mc + I] = (TO)(TI(0.25) * s);
}

// psi^{k+1}: (phi - phi^k)/s (scheme 1, eq. discrete_1_b) or
// (2/s)(phi - phi^k) - psi^k (scheme 2, eq. discrete_2_b); in place on psi.
// phi is also copied to phi_out (the caller's phi^{k+1}).
template <int SCHEME>
__device__ __forceinline__ void psi_cell(double s, const double* __restrict__ phi,
                                         const double* __restrict__ phik, double* psi,
                                         double* phi_out, size_t q) {
    const double x = phi[q];
    if constexpr (SCHEME == 1) psi[q] = (x - phik[q]) / s;
    else psi[q] = (2.0 / s) * (x - phik[q]) - psi[q];
    phi_out[q] = x;
}

template <int SCHEME>
__global__ void __launch_bounds__(256) k_psi_update(size_t total, double s,
                                                    const double* __restrict__ phi,
                                                    const double* __restrict__ phik, double* psi,
                                                    double* phi_out) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    psi_cell<SCHEME>(s, phi, phik, psi, phi_out, q);
}

}  // namespace mpfc
