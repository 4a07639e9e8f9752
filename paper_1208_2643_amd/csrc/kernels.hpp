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
// 1/x for x >= 1 (the determinant of the smoother's local system, 1 + a d +
// a b e_c with a, b, e_c, d >= 0): the hardware reciprocal estimate refined by
// Newton steps e = 1 - x r, r += r e (two in FP64, one in FP32), within an
// ulp of the correctly rounded quotient and shorter than a division.
__device__ __forceinline__ double recip_ge1(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float recip_ge1(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
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
    T w = T(1);  // relaxation factor of the smoother's cell update (1: App. B)
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
    const T* pin = nullptr;        // pinning weight W on this level (Sec. 4.6), else null
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
    const T dm = (r2 + (d + b * ec) * r1 - b * r3) * recip_ge1(det);
    const T dx = r1 - a * dm;
    const T dk = r3 - ec * dx;
    F.phi[q] = x + op.w * dx;
    F.mu[q] += op.w * dm;
    F.ka[q] += op.w * dk;
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


}  // namespace mpfc
