// Learned initial guess: a small periodic convolutional network, inference
// and training kernels for gfx950 (BF16 operands on the matrix cores, FP32
// accumulation).
//
// The step's initial guess is free (each step has exactly one solution, Sec. 3
// unique-solvability theorems), so a predictor may supply it:
//   x0 = in_scale * phi^n, x1 = (phi^n - phi^{n-1}) / sigma1 and
//   x2 = (s psi^n - (phi^n - phi^{n-1})) / sigma1 (sigma1 = rms of the
//   difference; x1 = x2 = 0 when it vanishes; psi^n enters because the step
//   depends on it and, for the second-order scheme, it carries the run's
//   history, eq. discrete_2_b), four 3x3 periodic convolutions
//   3 -> 32 -> 32 -> 32 -> 1 with tanh-form GELU after the first three, and the
//   guess 2 phi^n - phi^{n-1} + c with c = out_scale * sigma1 * delta minus its
//   mean (the guess keeps the mass of the extrapolation).
//
// Layouts.  Activations are BF16 (stored as uint16 bit patterns), NHWC with
// 32 channels: act[(s * NP + p) * 32 + c], p = y * m + x.  Parameters are an
// FP32 vector in blob order (W1 [3][3][3][32], b1, W2 [3][3][32][32], b2, W3,
// b3, W4 [3][3][32], b4).  A convolution is a GEMM per tap with the output
// channels as M (two 16-row tiles), 16 pixels of a tile row as N and the input
// channels as K; its weight operand is kept in registers as per-lane fragments
// prepared from the FP32 master weights (k_cnn_prepare32 and its siblings).
// Layer 1 gathers its 27 taps x channels, each input split into a BF16 hi and
// lo part, into one K = 64 operand (im2col in LDS).  The forward layers and
// the backward data pass run on v_mfma_f32_16x16x32_bf16; the weight
// gradients (GEMMs over pixels) on v_mfma_f32_16x16x16bf16_1k.
//
// Operand layouts (lane l, g = l / 16, c = l % 16): K = 32: A[m = c][k = 8g +
// i], B[k = 8g + i][n = c]; K = 16: A[m = c][k = 4g + i], B[k = 4g + i][n = c];
// both D[m = 4g + i][n = c].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "step.hpp"

namespace mpfc {

typedef short cnn_v4s __attribute__((ext_vector_type(4)));
typedef float cnn_v4f __attribute__((ext_vector_type(4)));

constexpr int CNN_CH = 32;
constexpr int CNN_TILE = 16;
constexpr int CNN_HALO = 18;
constexpr int CNN_PX = 36;           // LDS stride of one pixel (32 channels + 4 pad)
constexpr int CNN_NFRAG32 = 18;      // K = 32 instruction: 9 taps x 2 M tiles
// parameter offsets in the FP32 vector (blob order, no header)
constexpr int CNN_CIN = 3;
constexpr int CNN_W1 = 0, CNN_B1 = 864, CNN_W2 = 896, CNN_B2 = 10112, CNN_W3 = 10144,
              CNN_B3 = 19360, CNN_W4 = 19392, CNN_B4 = 19680, CNN_NPARAM = 19681;
constexpr int CNN_K1H = 9 * CNN_CIN;     // layer-1 K of one (hi or lo) part
constexpr int CNN_SEG1 = CNN_K1H * 32 + 32;  // layer-1 gradient segment (W1, b1)
constexpr int CNN_SEG = 9 * 32 * 32 + 32;  // layers 2, 3 (W, b)
constexpr int CNN_SEG4 = 9 * 32 + 1;     // layer 4 (W4, b4)

// Fields of one sample: the guess reads phi^{n-1}, phi^n, psi^n; training also
// phi^{n+1}; `out` receives the guess (inference).
struct CnnSample {
    const double* pm1;
    const double* p0;
    const double* psi;
    const double* pp1;
    double* out;
};

// FP32 -> BF16 (hardware conversion: round to nearest even, NaN kept).
__device__ __forceinline__ uint16_t bf16_bits(float f) {
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// tanh-form GELU, evaluated through the identity (1 + tanh u) / 2 = 1 / (1 + e^{-2u}):
// gelu(x) = x s, s = 1 / (1 + e^{-2u}), u = sqrt(2/pi) (x + 0.044715 x^3);
// gelu'(x) = s + 2 x s (1 - s) u'(x).
__device__ __forceinline__ float gelu_sig(float x) {
    const float u = 0.7978845608028654f * (x + 0.044715f * x * x * x);
    return __builtin_amdgcn_rcpf(1.0f + __expf(-2.0f * u));
}
__device__ __forceinline__ float gelu_f(float x) { return x * gelu_sig(x); }
__device__ __forceinline__ float gelu_grad_f(float x) {
    const float s = gelu_sig(x);
    return s + 2.0f * x * s * (1.0f - s) * 0.7978845608028654f * (1.0f + 0.134145f * x * x);
}

// Halo tile (18 x 18 pixels, 32 channels) of an NHWC activation into LDS
// (pixel stride CNN_PX), periodic wrap.  Workgroups of 256 threads; each
// thread moves CNN_HREG pieces of 16 bytes (8 channels of a pixel), all loads
// issued before the first is waited for: the piece index is clamped (surplus
// loads of the last threads repeat a valid piece and are not stored), so no
// load sits behind a branch.
constexpr int CNN_HCH = CNN_HALO * CNN_HALO * 4;  // 16-byte pieces of a halo tile
constexpr int CNN_HREG = (CNN_HCH + 255) / 256;   // ... per thread
__device__ __forceinline__ void cnn_load_halo(const uint16_t* __restrict__ act, size_t base,
                                              int x0, int y0, int m, int n, uint16_t* lds) {
    const int t = threadIdx.x;
    uint4 v[CNN_HREG];
#pragma unroll
    for (int j = 0; j < CNN_HREG; ++j) {
        const int c = min(t + 256 * j, CNN_HCH - 1);
        const int pi = c >> 2, part = c & 3;
        const int ty = pi / CNN_HALO, tx = pi - ty * CNN_HALO;
        const int gy = (y0 + ty - 1) & (n - 1), gx = (x0 + tx - 1) & (m - 1);
        v[j] = *(const uint4*)(act + (base + (size_t)gy * m + gx) * CNN_CH + part * 8);
    }
#pragma unroll
    for (int j = 0; j < CNN_HREG; ++j) {
        const int c = t + 256 * j;
        if (c < CNN_HCH) {
            uint2* d = (uint2*)(lds + (c >> 2) * CNN_PX + (c & 3) * 8);
            d[0] = make_uint2(v[j].x, v[j].y);
            d[1] = make_uint2(v[j].z, v[j].w);
        }
    }
}

// Layer-1 inputs of an 18 x 18 halo tile as BF16 pairs (hi, lo = the BF16
// rounding of what hi leaves), so that the first layer sees its inputs to about
// 16 significant bits: xs[c] (hi) and xs[3 + c] (lo) for x0 = in_scale * phi^n,
// x1 = (phi^n - phi^{n-1}) * inv_sigma1, x2 = (s psi^n - (phi^n - phi^{n-1})) *
// inv_sigma1.
__device__ __forceinline__ void cnn_load_inputs(const CnnSample& S, double in_scale, double dt,
                                                double inv_sigma1, int x0, int y0, int m, int n,
                                                uint16_t (*xs)[CNN_HALO * CNN_HALO]) {
    // 256 threads, two pixels each (the second clamped and not stored), all
    // six loads issued before any is used
    constexpr int NPIX = CNN_HALO * CNN_HALO;
    double p0[2], pm[2], ps[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int t = min((int)threadIdx.x + 256 * j, NPIX - 1);
        const int ty = t / CNN_HALO, tx = t - ty * CNN_HALO;
        const int gy = (y0 + ty - 1) & (n - 1), gx = (x0 + tx - 1) & (m - 1);
        const size_t q = (size_t)gy * m + gx;
        p0[j] = S.p0[q];
        pm[j] = S.pm1[q];
        ps[j] = S.psi[q];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int t = threadIdx.x + 256 * j;
        if (t >= NPIX) continue;
        const double v0 = p0[j], d1 = v0 - pm[j];
        const float x[3] = {(float)(in_scale * v0), (float)(d1 * inv_sigma1),
                            (float)((dt * ps[j] - d1) * inv_sigma1)};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const uint16_t hi = bf16_bits(x[c]);
            xs[c][t] = hi;
            xs[3 + c][t] = bf16_bits(x[c] - bf16_val(hi));
        }
    }
}

// im2col value k of tile pixel (ty, tx): k = part * 27 + tap * 3 + channel for
// the hi (part 0) and lo (part 1) inputs, 0 for k >= 54.
constexpr int CNN_K1 = 64;        // layer-1 K (54 used), 4 chunks of 16
__device__ __forceinline__ uint16_t cnn_im2col(const uint16_t (*xs)[CNN_HALO * CNN_HALO], int k,
                                               int ty, int tx) {
    if (k >= 2 * CNN_K1H) return 0;
    const int part = k >= CNN_K1H ? 1 : 0, kk = k - CNN_K1H * part;
    const int tap = kk / 3, c = kk - 3 * tap, ky = tap / 3, kx = tap - 3 * ky;
    return xs[3 * part + c][(ty + ky) * CNN_HALO + tx + kx];
}

struct CnnConvArgs {
    int m, n;
    const uint16_t* in;        // NHWC input (layers 2, 3 forward; backward data)
    const CnnSample* smp;      // layer 1: fields of every sample
    const double* sc;          // per sample: inv_sigma1, sigma_out, inv_sigma_out, 0
    double in_scale, dt;
    const uint16_t* wfrag;     // weight fragments
    const float* bias;         // forward
    uint16_t* out;             // NHWC output
    uint16_t* zout;            // forward: pre-activations (nullable)
    const uint16_t* zprev;     // backward data: pre-activations of the layer below
};

enum { CNN_FWD = 0, CNN_BWD = 1 };

// One 3x3 convolution layer with 32 output channels on a 16 x 16 tile of one
// sample, on the K = 32 instruction (v_mfma_f32_16x16x32_bf16:
// A[m = l % 16][k = 8 (l / 16) + i], B[k = 8 (l / 16) + i][n = l % 16],
// D[m = 4 (l / 16) + i][n = l % 16]).  FWD: out = gelu(conv(in) + b) (and
// z = conv(in) + b when zout is set).  BWD (transposed, flipped weights):
// out = conv(in) * gelu'(zprev).  The halo
// tile's LDS pixel stride is CNN_PX32, so every lane reads the 8 channels of
// its B operand as one 16-byte access.  Grid (m / 16, n / 16, samples), 256
// threads; wave w computes rows 4w ... 4w + 3, the nine taps outside and the
// four rows inside (eight independent accumulation chains).
constexpr int CNN_PX32 = 40;
typedef __bf16 cnn_v8b __attribute__((ext_vector_type(8)));

template <int MODE>
__global__ void __launch_bounds__(256, 3) k_cnn_conv32(CnnConvArgs A) {
    constexpr int RW = 4;                      // rows per wave (8 measured slower)
    constexpr int TH = 4 * RW;                 // tile rows (four waves of RW rows)
    constexpr int HR = TH + 2;                 // halo rows
    constexpr int NPC = HR * CNN_HALO * 4;     // 16-byte pieces of the halo tile
    constexpr int NREG = (NPC + 255) / 256;
    __shared__ __align__(16) uint16_t lds[HR * CNN_HALO * CNN_PX32];
    const int m = A.m, n = A.n;
    const size_t NP = (size_t)m * n;
    const int s = blockIdx.z;
    const size_t base = (size_t)s * NP;
    const int x0 = blockIdx.x * CNN_TILE, y0 = blockIdx.y * TH;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int g = lane >> 4, c16 = lane & 15;
    cnn_v8b wf[CNN_NFRAG32];
#pragma unroll
    for (int f = 0; f < CNN_NFRAG32; ++f)
        wf[f] = __builtin_bit_cast(cnn_v8b, *(const uint4*)(A.wfrag + ((size_t)f * 64 + lane) * 8));
    {
        // halo pieces as in cnn_load_halo, stored with the 16-byte stride
        uint4 v[NREG];
#pragma unroll
        for (int j = 0; j < NREG; ++j) {
            const int c = min(t + 256 * j, NPC - 1);
            const int pi = c >> 2, part = c & 3;
            const int ty = pi / CNN_HALO, tx = pi - ty * CNN_HALO;
            const int gy = (y0 + ty - 1) & (n - 1), gx = (x0 + tx - 1) & (m - 1);
            v[j] = *(const uint4*)(A.in + (base + (size_t)gy * m + gx) * CNN_CH + part * 8);
        }
#pragma unroll
        for (int j = 0; j < NREG; ++j) {
            const int c = t + 256 * j;
            if (c < NPC) *(uint4*)(lds + (c >> 2) * CNN_PX32 + (c & 3) * 8) = v[j];
        }
    }
    __syncthreads();
    cnn_v4f acc[RW][2];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        acc[r][0] = cnn_v4f{0.f, 0.f, 0.f, 0.f};
        acc[r][1] = cnn_v4f{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int ky = tap / 3, kx = tap - 3 * (tap / 3);
        cnn_v8b b[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r)
            b[r] = __builtin_bit_cast(
                cnn_v8b,
                *(const uint4*)(lds + ((wave * RW + r + ky) * CNN_HALO + c16 + kx) * CNN_PX32 + 8 * g));
#pragma unroll
        for (int r = 0; r < RW; ++r)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
                acc[r][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[tap * 2 + mt], b[r],
                                                                     acc[r][mt], 0, 0, 0);
    }
    // epilogue: lane holds channels 16 mt + 4g .. + 3 of pixel (row, c16)
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int row = wave * RW + r;
        const size_t q = base + (size_t)(y0 + row) * m + x0 + c16;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            const int co = mt * 16 + 4 * g;
            uint16_t o[4];
            if constexpr (MODE == CNN_FWD) {
                uint16_t zb[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float z = acc[r][mt][i] + A.bias[co + i];
                    zb[i] = bf16_bits(z);
                    o[i] = bf16_bits(gelu_f(z));
                }
                if (A.zout)
                    *(uint2*)(A.zout + q * CNN_CH + co) =
                        make_uint2((uint32_t)zb[0] | ((uint32_t)zb[1] << 16),
                                   (uint32_t)zb[2] | ((uint32_t)zb[3] << 16));
            } else {
                const uint2 zp = *(const uint2*)(A.zprev + q * CNN_CH + co);
                const uint16_t zv[4] = {(uint16_t)(zp.x & 0xffff), (uint16_t)(zp.x >> 16),
                                        (uint16_t)(zp.y & 0xffff), (uint16_t)(zp.y >> 16)};
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    o[i] = bf16_bits(acc[r][mt][i] * gelu_grad_f(bf16_val(zv[i])));
            }
            *(uint2*)(A.out + q * CNN_CH + co) =
                make_uint2((uint32_t)o[0] | ((uint32_t)o[1] << 16),
                           (uint32_t)o[2] | ((uint32_t)o[3] << 16));
        }
    }
}

// First layer (3 inputs as BF16 hi and lo parts -> 32 channels) on the K = 32
// instruction: the 27 taps x inputs of both parts (k = part * 27 + tap * 3 +
// input, zero from 54 to 63) are gathered into an im2col row per pixel (LDS
// pixel stride CNN_PX1_32, so a lane's 8 consecutive k are one 16-byte
// access) and contracted in two K = 32 chunks.
constexpr int CNN_PX1_32 = 72;
__global__ void __launch_bounds__(256) k_cnn_conv1_32(CnnConvArgs A) {
    __shared__ __align__(16) uint16_t lds[CNN_TILE * CNN_TILE * CNN_PX1_32];
    __shared__ uint16_t xs[6][CNN_HALO * CNN_HALO];
    const int m = A.m, n = A.n;
    const size_t NP = (size_t)m * n;
    const int s = blockIdx.z;
    const size_t base = (size_t)s * NP;
    const int x0 = blockIdx.x * CNN_TILE, y0 = blockIdx.y * CNN_TILE;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int g = lane >> 4, c16 = lane & 15;
    cnn_v8b wf[4];  // (kc, mt) = (f >> 1, f & 1)
#pragma unroll
    for (int f = 0; f < 4; ++f)
        wf[f] = __builtin_bit_cast(cnn_v8b, *(const uint4*)(A.wfrag + ((size_t)f * 64 + lane) * 8));
    const CnnSample S = A.smp[s];
    cnn_load_inputs(S, A.in_scale, A.dt, A.sc[4 * s + 0], x0, y0, m, n, xs);
    __syncthreads();
    {
        const int ty = t >> 4, tx = t & 15;
#pragma unroll
        for (int k = 0; k < CNN_K1; ++k) lds[t * CNN_PX1_32 + k] = cnn_im2col(xs, k, ty, tx);
    }
    __syncthreads();
    cnn_v4f acc[4][2];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        acc[r][0] = cnn_v4f{0.f, 0.f, 0.f, 0.f};
        acc[r][1] = cnn_v4f{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int kc = 0; kc < 2; ++kc)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const cnn_v8b b = __builtin_bit_cast(
                cnn_v8b,
                *(const uint4*)(lds + ((wave * 4 + r) * CNN_TILE + c16) * CNN_PX1_32 + kc * 32 + 8 * g));
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
                acc[r][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[kc * 2 + mt], b, acc[r][mt],
                                                                     0, 0, 0);
        }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const size_t q = base + (size_t)(y0 + wave * 4 + r) * m + x0 + c16;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            const int co = mt * 16 + 4 * g;
            uint16_t o[4], zb[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float z = acc[r][mt][i] + A.bias[co + i];
                zb[i] = bf16_bits(z);
                o[i] = bf16_bits(gelu_f(z));
            }
            if (A.zout)
                *(uint2*)(A.zout + q * CNN_CH + co) =
                    make_uint2((uint32_t)zb[0] | ((uint32_t)zb[1] << 16),
                               (uint32_t)zb[2] | ((uint32_t)zb[3] << 16));
            *(uint2*)(A.out + q * CNN_CH + co) =
                make_uint2((uint32_t)o[0] | ((uint32_t)o[1] << 16),
                           (uint32_t)o[2] | ((uint32_t)o[3] << 16));
        }
    }
}

struct CnnOutArgs {
    int m, n;
    const uint16_t* in;        // a3 (NHWC)
    const CnnSample* smp;
    const double* sc;
    const uint16_t* w4frag;    // output-layer weights as K = 32 fragments (k_cnn_prepare_out32)
    const float* b4;
    float* gd;                 // training: d loss / d delta
    double* part;              // per block and sample: sum of the correction / of err^2
    double gscale;             // training: 2 / (pixels of the batch)
};

// Output layer (32 -> 1) on a 16 x 16 tile.
// Inference: guess = 2 phi^n - phi^{n-1} + sigma_out * delta into smp.out and
// the block's sum of the correction.  Training: err = delta - target,
// gd = gscale * err and the block's sum of err^2.  part[blk * samples + s].
// It runs on the K = 32 instruction: M = 16 rows of which only row 0 (the one
// output channel) has weights, N = 16 pixels of a tile row, K = the 32
// channels of a tap; the products of BF16 values are exact in FP32, so only
// the order of the FP32 additions differs from a sum over taps and channels.
// The halo tile is read as in k_cnn_conv32; lanes 0-15 of each wave hold the
// row's 16 outputs (D[0][n]).
template <bool TRAIN>
__global__ void __launch_bounds__(256) k_cnn_out32(CnnOutArgs A) {
    __shared__ __align__(16) uint16_t lds[CNN_HALO * CNN_HALO * CNN_PX32];
    __shared__ double red[4];
    const int m = A.m, n = A.n;
    const size_t NP = (size_t)m * n;
    const int s = blockIdx.z;
    const size_t base = (size_t)s * NP;
    const int x0 = blockIdx.x * CNN_TILE, y0 = blockIdx.y * CNN_TILE;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int g = lane >> 4, c16 = lane & 15;
    cnn_v8b wf[9];
#pragma unroll
    for (int f = 0; f < 9; ++f)
        wf[f] = __builtin_bit_cast(cnn_v8b, *(const uint4*)(A.w4frag + ((size_t)f * 64 + lane) * 8));
    {
        uint4 v[CNN_HREG];
#pragma unroll
        for (int j = 0; j < CNN_HREG; ++j) {
            const int c = min(t + 256 * j, CNN_HCH - 1);
            const int pi = c >> 2, part = c & 3;
            const int ty = pi / CNN_HALO, tx = pi - ty * CNN_HALO;
            const int gy = (y0 + ty - 1) & (n - 1), gx = (x0 + tx - 1) & (m - 1);
            v[j] = *(const uint4*)(A.in + (base + (size_t)gy * m + gx) * CNN_CH + part * 8);
        }
#pragma unroll
        for (int j = 0; j < CNN_HREG; ++j) {
            const int c = t + 256 * j;
            if (c < CNN_HCH) *(uint4*)(lds + (c >> 2) * CNN_PX32 + (c & 3) * 8) = v[j];
        }
    }
    __syncthreads();
    cnn_v4f acc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = cnn_v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int ky = tap / 3, kx = tap - 3 * (tap / 3);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const cnn_v8b b = __builtin_bit_cast(
                cnn_v8b,
                *(const uint4*)(lds + ((wave * 4 + r + ky) * CNN_HALO + c16 + kx) * CNN_PX32 + 8 * g));
            acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[tap], b, acc[r], 0, 0, 0);
        }
    }
    const CnnSample S = A.smp[s];
    double sum = 0.0;
    if (g == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float d = acc[r][0] + A.b4[0];
            const size_t q = (size_t)(y0 + wave * 4 + r) * m + x0 + c16;
            if constexpr (!TRAIN) {
                const double corr = A.sc[4 * s + 1] * (double)d;
                S.out[q] = 2.0 * S.p0[q] - S.pm1[q] + corr;
                sum += corr;
            } else {
                const double tv = (S.pp1[q] - 2.0 * S.p0[q] + S.pm1[q]) * A.sc[4 * s + 2];
                const double err = (double)d - tv;
                A.gd[base + q] = (float)(A.gscale * err);
                sum += err * err;
            }
        }
    }
    const double bs = block_sum<256>(sum, red);
    if (t == 0) A.part[(size_t)(blockIdx.y * gridDim.x + blockIdx.x) * gridDim.z + s] = bs;
}

// The one sample of a step's learned guess: the caller's arrays from `io`,
// the guess into `out`.
__global__ void k_cnn_sample_io(CnnSample* smp, const StepIO* __restrict__ io, double* out) {
    if (threadIdx.x == 0) smp[0] = CnnSample{io->phi_nm1, io->phi_n, io->psi, nullptr, out};
}

// Per-sample scale factors from the sums of (phi^n - phi^{n-1})^2: one
// workgroup per sample s adds the per-block shares part[b * samples + s] over
// the nblk blocks in a fixed order, then sigma1 = rms of the difference.
template <int NT>
__global__ void __launch_bounds__(NT) k_cnn_scales_sum(const double* __restrict__ part, int nblk,
                                                       double npix, double out_scale, double* sc) {
    __shared__ double red[NT / 64];
    const int s = blockIdx.x, samples = gridDim.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += NT) acc += part[(size_t)b * samples + s];
    const double tot = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) {
        const double sig = sqrt(tot / npix);
        const double so = out_scale * sig;
        sc[4 * s + 0] = sig > 0.0 ? 1.0 / sig : 0.0;
        sc[4 * s + 1] = so;
        sc[4 * s + 2] = so > 0.0 ? 1.0 / so : 0.0;
        sc[4 * s + 3] = 0.0;
    }
}

// part[blk * samples + s] = block's share of sum (phi^n - phi^{n-1})^2 of sample s.
template <int NT>
__global__ void __launch_bounds__(NT) k_cnn_sigma(const CnnSample* __restrict__ smp, size_t npix,
                                                  double* part) {
    __shared__ double red[NT / 64];
    const int s = blockIdx.y;
    const CnnSample S = smp[s];
    double acc = 0.0;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < npix; q += (size_t)gridDim.x * NT) {
        const double d = S.p0[q] - S.pm1[q];
        acc += d * d;
    }
    const double bs = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * gridDim.y + s] = bs;
}

// Mean correction of the guesses: out -= sums[s] / npix.
__global__ void __launch_bounds__(256) k_cnn_shift(const CnnSample* __restrict__ smp, size_t npix,
                                                   const double* __restrict__ sums) {
    const int s = blockIdx.y;
    const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= npix) return;
    smp[s].out[q] -= sums[s] / (double)npix;
}

struct CnnOutBwdArgs {
    int m, n;
    const float* gd;           // d loss / d delta
    const float* w4;
    const uint16_t* z3;        // pre-activations of layer 3
    uint16_t* out;             // d loss / d z3
};

// dz3[p][c] = gelu'(z3[p][c]) * sum_tap w4[tap][c] gd[p - offset(tap)].
__global__ void __launch_bounds__(256) k_cnn_out_bwd(CnnOutBwdArgs A) {
    __shared__ float gs[CNN_HALO * CNN_HALO];
    __shared__ float w4s[9 * CNN_CH];
    const int m = A.m, n = A.n;
    const size_t NP = (size_t)m * n;
    const int s = blockIdx.z;
    const int x0 = blockIdx.x * CNN_TILE, y0 = blockIdx.y * CNN_TILE;
    for (int k = threadIdx.x; k < 9 * CNN_CH; k += 256) w4s[k] = A.w4[k];
    for (int t = threadIdx.x; t < CNN_HALO * CNN_HALO; t += 256) {
        const int ty = t / CNN_HALO, tx = t - ty * CNN_HALO;
        const int gy = (y0 + ty - 1) & (n - 1), gx = (x0 + tx - 1) & (m - 1);
        gs[t] = A.gd[(size_t)s * NP + (size_t)gy * m + gx];
    }
    __syncthreads();
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    float gn[9];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int ky = tap / 3, kx = tap - 3 * ky;
        gn[tap] = gs[(ty + 2 - ky) * CNN_HALO + tx + 2 - kx];
    }
    const size_t q = (size_t)s * NP + (size_t)(y0 + ty) * m + x0 + tx;
    for (int c = 0; c < CNN_CH; c += 4) {
        const uint2 zp = *(const uint2*)(A.z3 + q * CNN_CH + c);
        const uint16_t zv[4] = {(uint16_t)(zp.x & 0xffff), (uint16_t)(zp.x >> 16),
                                (uint16_t)(zp.y & 0xffff), (uint16_t)(zp.y >> 16)};
        uint16_t o[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float a = 0.f;
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) a += w4s[tap * CNN_CH + c + i] * gn[tap];
            o[i] = bf16_bits(a * gelu_grad_f(bf16_val(zv[i])));
        }
        *(uint2*)(A.out + q * CNN_CH + c) = make_uint2((uint32_t)o[0] | ((uint32_t)o[1] << 16),
                                                      (uint32_t)o[2] | ((uint32_t)o[3] << 16));
    }
}

struct CnnWgradArgs {
    int m, n, samples;
    const uint16_t* in;        // a_{L-1} (layers 2, 3)
    const CnnSample* smp;      // layer 1
    const double* sc;
    double in_scale, dt;
    const uint16_t* dz;        // d loss / d z_L
    float* part;               // [block][segment]
};

// Weight and bias gradients of a 32-output convolution layer:
// dW[tap][ci][co] = sum_p a[p + offset(tap)][ci] dz[p][co], db[co] = sum_p dz[p][co],
// as MFMA GEMMs over the pixels (K) of 16 x 16 tiles; every block loops over
// tiles and writes its partial sums (reduced in a fixed order by k_cnn_reduce).
// Both operands are staged in LDS with the pixel index fastest.
template <bool IM2COL>
__global__ void __launch_bounds__(256) k_cnn_wgrad(CnnWgradArgs A) {
    constexpr int AR = IM2COL ? CNN_TILE : CNN_HALO;   // rows of the A tile
    constexpr int RS = 20;                             // LDS row stride (pixels)
    constexpr int NCB = IM2COL ? 1 : 9;                // (tap, mt, nt) combos per wave
    constexpr int SEG = IM2COL ? CNN_SEG1 : CNN_SEG;
    __shared__ __align__(16) uint16_t la[32 * AR * RS];
    __shared__ __align__(16) uint16_t lb[32 * CNN_TILE * RS];
    __shared__ uint16_t xs[IM2COL ? 6 : 1][IM2COL ? CNN_HALO * CNN_HALO : 1];
    const int m = A.m, n = A.n;
    const size_t NP = (size_t)m * n;
    const int tx_n = m / CNN_TILE, ty_n = n / CNN_TILE;
    const int ntiles = tx_n * ty_n * A.samples;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c16 = lane & 15;
    cnn_v4f acc[NCB];
#pragma unroll
    for (int j = 0; j < NCB; ++j) acc[j] = cnn_v4f{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;
    for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const int s = tl / (tx_n * ty_n);
        const int rem = tl - s * tx_n * ty_n;
        const int by = rem / tx_n, bx = rem - by * tx_n;
        const int x0 = bx * CNN_TILE, y0 = by * CNN_TILE;
        __syncthreads();  // previous tile's LDS reads are done
        if constexpr (IM2COL) {
            cnn_load_inputs(A.smp[s], A.in_scale, A.dt, A.sc[4 * s + 0], x0, y0, m, n, xs);
            __syncthreads();
            const int t = threadIdx.x, ty = t >> 4, tx = t & 15;
            // the weight gradient takes the hi parts of the inputs (rows k < 27)
            for (int k = 0; k < 32; ++k)
                la[(k * CNN_TILE + ty) * RS + tx] = k < CNN_K1H ? cnn_im2col(xs, k, ty, tx) : (uint16_t)0;
        } else {
            for (int c = threadIdx.x; c < CNN_HALO * CNN_HALO * 4; c += 256) {
                const int pi = c >> 2, part = c & 3;
                const int ty = pi / CNN_HALO, tx = pi - ty * CNN_HALO;
                const int gy = (y0 + ty - 1) & (n - 1), gx = (x0 + tx - 1) & (m - 1);
                const uint4 v = *(const uint4*)(A.in + ((size_t)s * NP + (size_t)gy * m + gx) * CNN_CH + part * 8);
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    la[((part * 8 + j) * CNN_HALO + ty) * RS + tx] =
                        (uint16_t)((w[j >> 1] >> ((j & 1) * 16)) & 0xffff);
            }
        }
        for (int c = threadIdx.x; c < CNN_TILE * CNN_TILE * 4; c += 256) {
            const int pi = c >> 2, part = c & 3;
            const int ty = pi >> 4, tx = pi & 15;
            const uint4 v = *(const uint4*)(A.dz + ((size_t)s * NP + (size_t)(y0 + ty) * m + x0 + tx) * CNN_CH + part * 8);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 8; ++j)
                lb[((part * 8 + j) * CNN_TILE + ty) * RS + tx] = (uint16_t)((w[j >> 1] >> ((j & 1) * 16)) & 0xffff);
        }
        __syncthreads();
        if (threadIdx.x < 32) {
            float sb = 0.f;
            for (int y = 0; y < CNN_TILE; ++y)
                for (int x = 0; x < CNN_TILE; ++x) sb += bf16_val(lb[(threadIdx.x * CNN_TILE + y) * RS + x]);
            bacc += sb;
        }
        for (int y = 0; y < CNN_TILE; ++y) {
#pragma unroll
            for (int j = 0; j < NCB; ++j) {
                const int cb = wave * NCB + j;
                int tap, mt, nt;
                if constexpr (IM2COL) { tap = 0; mt = cb >> 1; nt = cb & 1; }
                else { tap = cb >> 2; mt = (cb >> 1) & 1; nt = cb & 1; }
                const int ky = tap / 3, kx = tap - 3 * ky;
                const int row = mt * 16 + c16;
                cnn_v4s a;
                const uint16_t* pa = la + (row * AR + y + (IM2COL ? 0 : ky)) * RS + 4 * g + (IM2COL ? 0 : kx);
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = (short)pa[i];
                const cnn_v4s b = *(const cnn_v4s*)(lb + ((nt * 16 + c16) * CNN_TILE + y) * RS + 4 * g);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[j], 0, 0, 0);
            }
        }
    }
    float* out = A.part + (size_t)blockIdx.x * SEG;
#pragma unroll
    for (int j = 0; j < NCB; ++j) {
        const int cb = wave * NCB + j;
        int tap, mt, nt;
        if constexpr (IM2COL) { tap = 0; mt = cb >> 1; nt = cb & 1; }
        else { tap = cb >> 2; mt = (cb >> 1) & 1; nt = cb & 1; }
        const int co = nt * 16 + c16;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ci = mt * 16 + 4 * g + i;
            if constexpr (IM2COL) {
                if (ci < CNN_K1H) out[ci * CNN_CH + co] = acc[j][i];
            } else {
                out[(tap * CNN_CH + ci) * CNN_CH + co] = acc[j][i];
            }
        }
    }
    if (threadIdx.x < 32) out[SEG - 32 + threadIdx.x] = bacc;
}

struct CnnW4Args {
    int m, n, samples;
    const uint16_t* in;        // a3
    const float* gd;
    float* part;               // [block][CNN_SEG4]
};

// Gradients of the output layer: dW4[tap][c] = sum_p a3[p + offset(tap)][c] gd[p],
// db4 = sum_p gd[p]; per-block partial sums over a strided set of tiles.
__global__ void __launch_bounds__(256) k_cnn_w4grad(CnnW4Args A) {
    __shared__ __align__(16) uint16_t lds[CNN_HALO * CNN_HALO * CNN_PX];
    __shared__ float gs[CNN_TILE * CNN_TILE];
    const int m = A.m, n = A.n;
    const size_t NP = (size_t)m * n;
    const int tx_n = m / CNN_TILE, ty_n = n / CNN_TILE;
    const int ntiles = tx_n * ty_n * A.samples;
    float acc[2] = {0.f, 0.f};
    for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const int s = tl / (tx_n * ty_n);
        const int rem = tl - s * tx_n * ty_n;
        const int by = rem / tx_n, bx = rem - by * tx_n;
        const int x0 = bx * CNN_TILE, y0 = by * CNN_TILE;
        __syncthreads();
        cnn_load_halo(A.in, (size_t)s * NP, x0, y0, m, n, lds);
        {
            const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
            gs[threadIdx.x] = A.gd[(size_t)s * NP + (size_t)(y0 + ty) * m + x0 + tx];
        }
        __syncthreads();
        for (int k = 0; k < 2; ++k) {
            const int o = threadIdx.x + 256 * k;
            if (o >= CNN_SEG4) break;
            float sum = 0.f;
            if (o < 9 * CNN_CH) {
                const int tap = o / CNN_CH, c = o - tap * CNN_CH;
                const int ky = tap / 3, kx = tap - 3 * ky;
                for (int y = 0; y < CNN_TILE; ++y)
                    for (int x = 0; x < CNN_TILE; ++x)
                        sum += bf16_val(lds[((y + ky) * CNN_HALO + x + kx) * CNN_PX + c]) * gs[y * CNN_TILE + x];
            } else {
                for (int p = 0; p < CNN_TILE * CNN_TILE; ++p) sum += gs[p];
            }
            acc[k] += sum;
        }
    }
    for (int k = 0; k < 2; ++k) {
        const int o = threadIdx.x + 256 * k;
        if (o < CNN_SEG4) A.part[(size_t)blockIdx.x * CNN_SEG4 + o] = acc[k];
    }
}

// out[i] = sum over blocks b (in order) of part[b * seg + i].
__global__ void __launch_bounds__(256) k_cnn_reduce(const float* __restrict__ part, int nblk,
                                                    int seg, float* out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= seg) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * seg + i];
    out[i] = s;
}

// Adam on the FP32 master parameters (Kingma and Ba, 2015); c1, c2 are the
// bias corrections 1 / (1 - beta^t).
__global__ void __launch_bounds__(256) k_cnn_adam(float* theta, const float* __restrict__ grad,
                                                  float* mom, float* vel, int count, float lr,
                                                  float b1, float b2, float eps, float c1,
                                                  float c2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const float gr = grad[i];
    const float m1 = b1 * mom[i] + (1.f - b1) * gr;
    const float v1 = b2 * vel[i] + (1.f - b2) * gr * gr;
    mom[i] = m1;
    vel[i] = v1;
    theta[i] -= lr * (m1 * c1) / (sqrtf(v1 * c2) + eps);
}

// Per-lane weight fragments (BF16) from the FP32 parameters:
//   f1: layer 1, [kc][mt][lane][4], A[co][k] = W1[tap][c][co] for k = part * 27 + tap * 3 + c
//       (the same weight for the hi and lo part of an input; 0 for k >= 54);
//   f2, f3: layers 2, 3 forward, [tap][kc][mt][lane][4], A[co][ci] = W[tap][ci][co];
//   r2, r3: backward data, A[co'][ci'] = W[8 - tap][co'][ci'] (flipped taps, swapped channels);
//   w4: output-layer weights rounded to BF16 (as floats).
// Weight operands for the K = 32 instruction, prepared from the FP32 master
// weights after every change (load, Adam step).
struct CnnFrags {
    uint16_t* x1;   // layer 1 (k_cnn_conv1_32): 2 K chunks x 2 M tiles
    uint16_t* x2;   // layers 2, 3 forward (k_cnn_conv32<CNN_FWD>): 9 taps x 2 M tiles
    uint16_t* x3;
    uint16_t* r2;   // layers 2, 3 backward data (k_cnn_conv32<CNN_BWD>): flipped, transposed
    uint16_t* r3;
    uint16_t* x4;   // output layer (k_cnn_out32): 9 fragments, row 0 only
    float* w4;      // output layer, BF16-rounded FP32 values (k_cnn_out_bwd)
};

// Weight fragments of layers 2 and 3: fragment f = tap * 2 + mt, lane l,
// element i at ((f * 64 + l) * 8 + i) holds, with a = 16 mt + l % 16 and
// b = 8 (l / 16) + i, forward W[tap][ci = b][co = a]; backward data the
// flipped, transposed W[8 - tap][ci = a][co = b].
__global__ void __launch_bounds__(256) k_cnn_prepare32(const float* __restrict__ th, CnnFrags F) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    constexpr int NX = CNN_NFRAG32 * 64 * 8;
    if (e >= 4 * NX) return;
    const int which = e / NX, r = e - which * NX;   // x2, x3, r2, r3
    const int f = r >> 9, lane = (r >> 3) & 63, i = r & 7;
    const int tap = f >> 1, mt = f & 1;
    const int a = mt * 16 + (lane & 15), b = 8 * (lane >> 4) + i;
    const int base = (which & 1) ? CNN_W3 : CNN_W2;
    uint16_t* dst = which == 0 ? F.x2 : which == 1 ? F.x3 : which == 2 ? F.r2 : F.r3;
    const float v = which < 2 ? th[base + (tap * CNN_CH + b) * CNN_CH + a]
                              : th[base + ((8 - tap) * CNN_CH + a) * CNN_CH + b];
    dst[r] = bf16_bits(v);
}

// Layer-1 fragments for k_cnn_conv1_32: fragment f = kc * 2 + mt, lane l,
// element i holds W1 at k = 32 kc + 8 (l / 16) + i (both BF16 parts of an
// input share its weight; zero for k >= 54), co = 16 mt + l % 16.
__global__ void __launch_bounds__(256) k_cnn_prepare1_32(const float* __restrict__ th, CnnFrags F) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= 4 * 64 * 8) return;
    const int f = e >> 9, lane = (e >> 3) & 63, i = e & 7;
    const int kc = f >> 1, mt = f & 1;
    const int co = mt * 16 + (lane & 15), k = kc * 32 + 8 * (lane >> 4) + i;
    F.x1[e] = k < 2 * CNN_K1H ? bf16_bits(th[CNN_W1 + (k % CNN_K1H) * CNN_CH + co]) : (uint16_t)0;
}

// Output-layer fragments for k_cnn_out32: fragment tap, lane l, element i holds
// W4[tap][ci = 8 (l / 16) + i] in row m = l % 16 = 0, zero in the other rows.
__global__ void __launch_bounds__(256) k_cnn_prepare_out32(const float* __restrict__ th, CnnFrags F) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= 9 * 64 * 8) return;
    const int tap = e >> 9, lane = (e >> 3) & 63, i = e & 7;
    const int ci = 8 * (lane >> 4) + i;
    F.x4[e] = (lane & 15) == 0 ? bf16_bits(th[CNN_W4 + tap * CNN_CH + ci]) : (uint16_t)0;
}

// Output-layer weights rounded to BF16 (kept as FP32 values) for k_cnn_out_bwd.
__global__ void __launch_bounds__(256) k_cnn_prepare(const float* __restrict__ th, CnnFrags F) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < 9 * CNN_CH) F.w4[e] = bf16_val(bf16_bits(th[CNN_W4 + e]));
}

// Candidates of the step's initial guess, the learned one in copy 0 and the
// extrapolated one in copy 1: per-block sums of the first residual component
// squared of both in one pass (part[b] for copy 0, part[gridDim.x + b] for
// copy 1; the completion makes the other components vanish).
template <int NT>
__global__ void __launch_bounds__(NT) k_cnn_resnorm2(Fields<double> A, Fields<double> B,
                                                     LevelOp<double> op, Grid g, double* part) {
    __shared__ double red[2][NT / 64];  // one per sum: thread 0 reads them after the barrier
    double a2 = 0.0, b2 = 0.0;
    const size_t total = (size_t)g.m * g.n;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        int i, j;
        cell_of(q, g, i, j);
        const double ra = A.f1[q] - (A.phi[q] - op.c * (nsum(A.mu, i, j, g) - 4.0 * A.mu[q]) * op.ih2);
        const double rb = B.f1[q] - (B.phi[q] - op.c * (nsum(B.mu, i, j, g) - 4.0 * B.mu[q]) * op.ih2);
        a2 += ra * ra;
        b2 += rb * rb;
    }
    const double sa = block_sum<NT>(a2, red[0]);
    const double sb = block_sum<NT>(b2, red[1]);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = sa;
        part[gridDim.x + blockIdx.x] = sb;
    }
}

// The choice, one workgroup: r2[0], r2[1] = the two candidates' sums (fixed
// order); the learned guess is used when its sum is the smaller one (a NaN
// network falls back); counts[0] counts the steps that used it, counts[1]
// the fallbacks; part[0] receives the kept guess's sum (the step's first norm).
template <int NT>
__global__ void __launch_bounds__(NT) k_cnn_decide(double* part, int nblk, double* r2,
                                                   unsigned long long* counts) {
    __shared__ double red[2][NT / 64];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nblk; k += NT) {
        a += part[k];
        b += part[nblk + k];
    }
    const double sa = block_sum<NT>(a, red[0]);
    const double sb = block_sum<NT>(b, red[1]);
    if (threadIdx.x == 0) {
        const bool use = sa < sb;
        r2[0] = sa;
        r2[1] = sb;
        counts[use ? 0 : 1] += 1ull;
        part[0] = use ? sa : sb;
    }
}

// Fallback: the extrapolated guess (copy 1) over the learned one (copy 0)
// when k_cnn_decide did not keep the learned one.
__global__ void __launch_bounds__(256) k_cnn_pick(const double* __restrict__ r2, size_t total,
                                                  double* u0a, double* u0b, double* u0c,
                                                  const double* __restrict__ u1a,
                                                  const double* __restrict__ u1b,
                                                  const double* __restrict__ u1c) {
    const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (r2[0] < r2[1] || q >= total) return;
    u0a[q] = u1a[q];
    u0b[q] = u1b[q];
    u0c[q] = u1c[q];
}

// Completion of the learned candidate's mu, with the correction's mean (sum
// csum[0] over the grid, times inv_npix) taken off its phi first, so the guess
// keeps the extrapolation's mass.  Each thread shifts its own cell only (kappa
// was formed before from the unshifted phi, whose Laplacian is the same).
template <int SCHEME>
__global__ void __launch_bounds__(256) k_cnn_complete_mu(Grid g, double ih2, double al,
                                                         double* phi,
                                                         const double* __restrict__ phik,
                                                         const double* __restrict__ ka,
                                                         const double* __restrict__ S2, double* mu,
                                                         const double* __restrict__ pin,
                                                         const double* __restrict__ csum,
                                                         double inv_npix) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.m || j >= g.n) return;
    const size_t q = at(i, j, g);
    const double x = phi[q] - csum[0] * inv_npix;
    phi[q] = x;
    complete_mu_at<SCHEME>(g, ih2, al, x, phik, ka, S2, mu, i, j, pin);
}

}  // namespace mpfc
