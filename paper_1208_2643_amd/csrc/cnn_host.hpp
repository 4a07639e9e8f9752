// Host side of the learned initial guess (included at the end of mpfc.hip):
// the network state shared by inference inside mpfc_step and by the trainer,
// and the C entry points.
#pragma once
#include "cnn.hpp"

struct mpfc_cnn_trainer;

namespace {

constexpr int CNN_BLOB_HEADER = 8;
constexpr int CNN_BLOB = CNN_BLOB_HEADER + CNN_NPARAM;

int cnn_check_blob(const float* blob, size_t count) {
    if (!blob) return fail(MPFC_EINVAL, "network blob is NULL");
    if (count != (size_t)CNN_BLOB) return fail(MPFC_EINVAL, "network blob has the wrong size");
    if ((int)blob[0] != 2 || (int)blob[1] != CNN_CIN || (int)blob[2] != CNN_CH || (int)blob[3] != 4)
        return fail(MPFC_EINVAL, "network blob header does not match (version 2, 3-32-32-32-1)");
    if (!std::isfinite(blob[4]) || !std::isfinite(blob[5]) || !(blob[6] > 0))
        return fail(MPFC_EINVAL, "network blob scales or time step are not valid");
    return MPFC_OK;
}

int cnn_check_grid(int m, int n) {
    if (!is_pow2(m) || !is_pow2(n) || m < CNN_TILE || n < CNN_TILE)
        return fail(MPFC_EINVAL, "the network needs power-of-two grids of at least 16 x 16");
    return MPFC_OK;
}

// Parameters, fragments and activations of the network for `B` samples of
// an m x n grid.  `train` adds what the backward pass and Adam need.
struct CnnNet {
    int m = 0, n = 0, B = 0;
    size_t NP = 0;
    bool train = false;
    double in_scale = 1, out_scale = 1, dt = 0;
    std::vector<void*> allocs;
    float* theta = nullptr;
    float *grad = nullptr, *mom = nullptr, *vel = nullptr;
    CnnFrags fr{};
    uint16_t* a[4] = {};      // activations (inference: a[1], a[2] ping-pong)
    uint16_t* z[4] = {};      // training: pre-activations
    uint16_t* dz[2] = {};
    float* gd = nullptr;
    CnnSample* d_smp = nullptr;
    CnnSample* h_smp = nullptr;  // pinned
    double* sc = nullptr;
    double* part = nullptr;      // [block][sample]
    double* sums = nullptr;      // [sample]
    double* h_sums = nullptr;    // pinned
    int nblk_sig = 0, nblk_out = 0;
    float* wpart = nullptr;
    int nblk_w = 0;
    int adam_t = 0;

    template <typename T>
    int dalloc(T** p, size_t count) {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, count * sizeof(T) + 64);
        if (e != hipSuccess) return fail(MPFC_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        allocs.push_back(q);
        *p = (T*)q;
        return MPFC_OK;
    }

    ~CnnNet() {
        for (void* p : allocs) (void)hipFree(p);
        if (h_smp) (void)hipHostFree(h_smp);
        if (h_sums) (void)hipHostFree(h_sums);
    }

    int init(int m_, int n_, int B_, bool train_) {
        m = m_; n = n_; B = B_; train = train_;
        NP = (size_t)m * n;
        const size_t act = (size_t)B * NP * CNN_CH;
        int rc = MPFC_OK;
        auto A = [&](auto** p, size_t cnt) { if (!rc) rc = dalloc(p, cnt); };
        A(&theta, CNN_NPARAM);
        A(&fr.x1, 4 * 64 * 8);
        A(&fr.x2, CNN_NFRAG32 * 64 * 8);
        A(&fr.x3, CNN_NFRAG32 * 64 * 8);
        A(&fr.r2, CNN_NFRAG32 * 64 * 8);
        A(&fr.r3, CNN_NFRAG32 * 64 * 8);
        A(&fr.x4, 9 * 64 * 8);
        A(&fr.w4, 9 * CNN_CH);
        if (train) {
            for (int l = 1; l <= 3; ++l) { A(&a[l], act); A(&z[l], act); }
            A(&dz[0], act);
            A(&dz[1], act);
            A(&gd, (size_t)B * NP);
            A(&grad, CNN_NPARAM);
            A(&mom, CNN_NPARAM);
            A(&vel, CNN_NPARAM);
            nblk_w = 512;
            A(&wpart, (size_t)nblk_w * CNN_SEG);
        } else {
            A(&a[1], act);
            A(&a[2], act);
            a[3] = a[1];
        }
        nblk_sig = (int)std::min<size_t>(256, (NP + 1023) / 1024);
        nblk_out = (int)((m / CNN_TILE) * (n / CNN_TILE));
        A(&d_smp, B);
        A(&sc, 4 * (size_t)B);
        A(&part, (size_t)B * std::max(nblk_sig, nblk_out));
        A(&sums, B);
        if (rc) return rc;
        if (hipHostMalloc((void**)&h_smp, B * sizeof(CnnSample), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&h_sums, B * sizeof(double), hipHostMallocDefault) != hipSuccess)
            return fail(MPFC_ENOMEM, "hipHostMalloc");
        if (train) {
            HIP_TRY(hipMemset(mom, 0, CNN_NPARAM * sizeof(float)));
            HIP_TRY(hipMemset(vel, 0, CNN_NPARAM * sizeof(float)));
        }
        return MPFC_OK;
    }

    void prepare(hipStream_t s) {
        hipLaunchKernelGGL(k_cnn_prepare, dim3((9 * CNN_CH + 255) / 256), dim3(256), 0, s, theta, fr);
        hipLaunchKernelGGL(k_cnn_prepare32, dim3(4 * CNN_NFRAG32 * 64 * 8 / 256), dim3(256), 0, s,
                           theta, fr);
        hipLaunchKernelGGL(k_cnn_prepare_out32, dim3(9 * 64 * 8 / 256), dim3(256), 0, s, theta, fr);
        hipLaunchKernelGGL(k_cnn_prepare1_32, dim3(4 * 64 * 8 / 256), dim3(256), 0, s, theta, fr);
    }

    int load(const float* blob, hipStream_t s) {
        in_scale = blob[4];
        out_scale = blob[5];
        dt = blob[6];
        HIP_TRY(hipMemcpyAsync(theta, blob + CNN_BLOB_HEADER, CNN_NPARAM * sizeof(float),
                               hipMemcpyHostToDevice, s));
        prepare(s);
        HIP_TRY(hipStreamSynchronize(s));
        adam_t = 0;
        return MPFC_OK;
    }

    int set_samples(hipStream_t s) {
        HIP_TRY(hipMemcpyAsync(d_smp, h_smp, B * sizeof(CnnSample), hipMemcpyHostToDevice, s));
        return MPFC_OK;
    }

    // A forward 32 -> 32 layer on the K = 32 instruction.
    void conv32(const CnnConvArgs& c, hipStream_t s) {
        hipLaunchKernelGGL((k_cnn_conv32<CNN_FWD>), dim3(m / CNN_TILE, n / CNN_TILE, B), dim3(256), 0,
                           s, c);
    }

    // Scales, three hidden layers and the output layer.  Inference writes the
    // guess into every sample's `out` and the sum of its correction into
    // `sums`; with `shift` the correction's mean is taken off there (the step
    // does that in the candidate's completion instead).  Training writes
    // d loss / d delta and leaves the per-sample sums of err^2 in `sums`.
    void forward(hipStream_t s, bool training, bool shift = true) {
        const dim3 tg(m / CNN_TILE, n / CNN_TILE, B), blk(256);
        hipLaunchKernelGGL((k_cnn_sigma<256>), dim3(nblk_sig, B), blk, 0, s, d_smp, NP, part);
        hipLaunchKernelGGL((k_cnn_scales_sum<256>), dim3(B), blk, 0, s, part, nblk_sig, (double)NP,
                           out_scale, sc);
        CnnConvArgs c{};
        c.m = m; c.n = n; c.smp = d_smp; c.sc = sc; c.in_scale = in_scale; c.dt = dt;
        c.wfrag = fr.x1; c.bias = theta + CNN_B1; c.out = a[1]; c.zout = training ? z[1] : nullptr;
        hipLaunchKernelGGL(k_cnn_conv1_32, tg, blk, 0, s, c);
        c.in = a[1]; c.wfrag = fr.x2; c.bias = theta + CNN_B2; c.out = a[2];
        c.zout = training ? z[2] : nullptr;
        conv32(c, s);
        c.in = a[2]; c.wfrag = fr.x3; c.bias = theta + CNN_B3; c.out = a[3];
        c.zout = training ? z[3] : nullptr;
        conv32(c, s);
        CnnOutArgs o{};
        o.m = m; o.n = n; o.in = a[3]; o.smp = d_smp; o.sc = sc; o.w4frag = fr.x4;
        o.b4 = theta + CNN_B4; o.gd = gd; o.part = part;
        o.gscale = 2.0 / ((double)B * (double)NP);
        if (training) {
            hipLaunchKernelGGL((k_cnn_out32<true>), tg, blk, 0, s, o);
            hipLaunchKernelGGL((k_partials_sum<256>), dim3(1), blk, 0, s, part, nblk_out, B, sums);
        } else {
            hipLaunchKernelGGL((k_cnn_out32<false>), tg, blk, 0, s, o);
            hipLaunchKernelGGL((k_partials_sum<256>), dim3(1), blk, 0, s, part, nblk_out, B, sums);
            if (shift)
                hipLaunchKernelGGL(k_cnn_shift, dim3((unsigned)((NP + 255) / 256), B), blk, 0, s,
                                   d_smp, NP, sums);
        }
    }

    void reduce(int seg, int off, hipStream_t s) {
        hipLaunchKernelGGL(k_cnn_reduce, dim3((seg + 255) / 256), dim3(256), 0, s, wpart, nblk_w, seg,
                           grad + off);
    }

    // Gradients of the loss of the last training forward pass into `grad`.
    void backward(hipStream_t s) {
        const dim3 tg(m / CNN_TILE, n / CNN_TILE, B), blk(256);
        CnnOutBwdArgs ob{m, n, gd, fr.w4, z[3], dz[0]};
        hipLaunchKernelGGL(k_cnn_out_bwd, tg, blk, 0, s, ob);
        CnnW4Args w4{m, n, B, a[3], gd, wpart};
        hipLaunchKernelGGL(k_cnn_w4grad, dim3(nblk_w), blk, 0, s, w4);
        reduce(CNN_SEG4, CNN_W4, s);
        CnnWgradArgs wg{};
        wg.m = m; wg.n = n; wg.samples = B; wg.smp = d_smp; wg.sc = sc; wg.in_scale = in_scale;
        wg.dt = dt;
        wg.part = wpart;
        wg.in = a[2]; wg.dz = dz[0];
        hipLaunchKernelGGL((k_cnn_wgrad<false>), dim3(nblk_w), blk, 0, s, wg);
        reduce(CNN_SEG, CNN_W3, s);
        CnnConvArgs c{};
        c.m = m; c.n = n; c.in = dz[0]; c.wfrag = fr.r3; c.zprev = z[2]; c.out = dz[1];
        hipLaunchKernelGGL((k_cnn_conv32<CNN_BWD>), tg, blk, 0, s, c);
        wg.in = a[1]; wg.dz = dz[1];
        hipLaunchKernelGGL((k_cnn_wgrad<false>), dim3(nblk_w), blk, 0, s, wg);
        reduce(CNN_SEG, CNN_W2, s);
        c.in = dz[1]; c.wfrag = fr.r2; c.zprev = z[1]; c.out = dz[0];
        hipLaunchKernelGGL((k_cnn_conv32<CNN_BWD>), tg, blk, 0, s, c);
        wg.dz = dz[0];
        hipLaunchKernelGGL((k_cnn_wgrad<true>), dim3(nblk_w), blk, 0, s, wg);
        reduce(CNN_SEG1, CNN_W1, s);
    }

    void adam(const mpfc_cnn_hparams& hp, hipStream_t s) {
        ++adam_t;
        const double c1 = 1.0 / (1.0 - std::pow((double)hp.beta1, adam_t));
        const double c2 = 1.0 / (1.0 - std::pow((double)hp.beta2, adam_t));
        hipLaunchKernelGGL(k_cnn_adam, dim3((CNN_NPARAM + 255) / 256), dim3(256), 0, s, theta, grad,
                           mom, vel, CNN_NPARAM, hp.lr, hp.beta1, hp.beta2, hp.eps, (float)c1,
                           (float)c2);
        prepare(s);
    }
};

void cnn_free(CnnNet* net) { delete net; }

}  // namespace

struct mpfc_cnn_trainer {
    CnnNet net;
    mpfc_cnn_hparams hp{};
    hipStream_t stream = nullptr;
};

namespace {

// Learned guess of one step into copy 0 of the finest level and its
// completion (kappa, mu); the step's source S is in place.  The step's phi^n,
// phi^{n-1} and psi^n are the caller's arrays in `io`.
int cnn_candidate(mpfc_ctx* C, const StepIO* io, hipStream_t s) {
    Level& F0 = C->L[0];
    const Grid g0 = F0.g;
    const double ih2 = 1.0 / (F0.h * F0.h);
    CnnNet& N = *C->cnn;
    hipLaunchKernelGGL(k_cnn_sample_io, dim3(1), dim3(64), 0, s, N.d_smp, io, F0.u[0][0]);
    N.forward(s, false, false);  // the correction's mean is taken off in the mu pass
    const double e = C->p.scheme == 1 ? 1.0 : 0.5;
    const double al = C->p.scheme == 1 ? C->alpha : 0.5 * C->alpha;
    const double inv_npix = 1.0 / (double)((size_t)C->m * C->n);
    hipLaunchKernelGGL(k_complete_kappa, grid2(C->m, C->n), B2, 0, s, g0, ih2, e, F0.u[0][0],
                       F0.f[2], F0.u[0][2]);
    if (C->p.scheme == 1)
        hipLaunchKernelGGL((k_cnn_complete_mu<1>), grid2(C->m, C->n), B2, 0, s, g0, ih2, al,
                           F0.u[0][0], C->phik, F0.u[0][2], F0.f[1], F0.u[0][1],
                           (const double*)nullptr, (const double*)N.sums, inv_npix);
    else
        hipLaunchKernelGGL((k_cnn_complete_mu<2>), grid2(C->m, C->n), B2, 0, s, g0, ih2, al,
                           F0.u[0][0], C->phik, F0.u[0][2], F0.f[1], F0.u[0][1],
                           (const double*)(C->pinned ? F0.pin : nullptr), (const double*)N.sums,
                           inv_npix);
    return MPFC_OK;
}

// Candidate choice: the first residual component of both completed
// candidates (the other two vanish by construction) in one pass, the choice
// in one workgroup, and the extrapolated guess (copy 1) copied over the
// learned one (copy 0) only when it has the smaller residual.
void cnn_choose(mpfc_ctx* C, hipStream_t s) {
    Level& F0 = C->L[0];
    const size_t total = (size_t)C->m * C->n;
    Fields<double> F[2];
    for (int k = 0; k < 2; ++k) {
        F[k].phi = F0.u[k][0]; F[k].mu = F0.u[k][1]; F[k].ka = F0.u[k][2];
        F[k].f1 = F0.f[0]; F[k].f2 = F0.f[1]; F[k].f3 = F0.f[2];
        F[k].phik = C->p.scheme == 2 ? C->phik : nullptr;
        F[k].base = nullptr;
        F[k].pin = C->pinned ? F0.pin : nullptr;
    }
    const unsigned nb = red_blocks(total);
    hipLaunchKernelGGL((k_cnn_resnorm2<NT>), dim3(nb), dim3(NT), 0, s, F[0], F[1],
                       level_op(C, F0), F0.g, C->part);
    hipLaunchKernelGGL((k_cnn_decide<NT>), dim3(1), dim3(NT), 0, s, C->part, (int)nb, C->cnn_r2,
                       C->cnn_counts);
    hipLaunchKernelGGL(k_cnn_pick, grid1(total), dim3(256), 0, s, C->cnn_r2, total, F0.u[0][0],
                       F0.u[0][1], F0.u[0][2], F0.u[1][0], F0.u[1][1], F0.u[1][2]);
}

}  // namespace

extern "C" {

int mpfc_cnn_blob_size(void) { return CNN_BLOB; }

int mpfc_cnn_load(mpfc_ctx* C, const float* blob, size_t count) {
    if (!C) return fail(MPFC_EINVAL, "ctx is NULL");
    int rc = cnn_check_blob(blob, count);
    if (!rc) rc = cnn_check_grid(C->m, C->n);
    if (rc) return rc;
    if (std::fabs(blob[6] - C->p.dt) > 1e-6 * C->p.dt)
        return fail(MPFC_EINVAL, "the network was trained for another time step");
    if (!C->cnn) {
        CnnNet* N = new (std::nothrow) CnnNet();
        if (!N) return fail(MPFC_ENOMEM, "host allocation failed");
        rc = N->init(C->m, C->n, 1, false);
        if (rc) { delete N; return rc; }
        C->cnn = N;
    }
    rc = C->cnn->load(blob, C->stream);
    if (rc) return rc;
    // the candidate's residual is computed once the context exists
    HIP_TRY(hipMemsetAsync(C->cnn_counts, 0, 2 * sizeof(unsigned long long), C->stream));
    HIP_TRY(hipStreamSynchronize(C->stream));
    return MPFC_OK;
}

int mpfc_cnn_counts(mpfc_ctx* C, long long* used, long long* fallbacks) {
    if (!C) return fail(MPFC_EINVAL, "ctx is NULL");
    unsigned long long h[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(h, C->cnn_counts, sizeof h, hipMemcpyDeviceToHost, C->stream));
    HIP_TRY(hipStreamSynchronize(C->stream));
    if (used) *used = (long long)h[0];
    if (fallbacks) *fallbacks = (long long)h[1];
    return MPFC_OK;
}

int mpfc_cnn_trainer_create(mpfc_cnn_trainer** out, int m, int n, int batch, const float* blob,
                            size_t count, const mpfc_cnn_hparams* hp, void* stream) {
    if (!out) return fail(MPFC_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = cnn_check_blob(blob, count);
    if (!rc) rc = cnn_check_grid(m, n);
    if (rc) return rc;
    if (batch < 1 || batch > 256) return fail(MPFC_EINVAL, "batch must be in [1, 256]");
    if ((long long)m * n * batch > (1LL << 26))
        return fail(MPFC_EINVAL, "batch too large (m n batch > 2^26 pixels)");
    if (!hp || !(hp->lr > 0) || !(hp->beta1 >= 0 && hp->beta1 < 1) ||
        !(hp->beta2 >= 0 && hp->beta2 < 1) || !(hp->eps > 0))
        return fail(MPFC_EINVAL, "invalid optimiser settings");
    mpfc_cnn_trainer* T = new (std::nothrow) mpfc_cnn_trainer();
    if (!T) return fail(MPFC_ENOMEM, "host allocation failed");
    T->hp = *hp;
    T->stream = (hipStream_t)stream;
    rc = T->net.init(m, n, batch, true);
    if (!rc) rc = T->net.load(blob, T->stream);
    if (rc) {
        delete T;
        return rc;
    }
    *out = T;
    return MPFC_OK;
}

void mpfc_cnn_trainer_destroy(mpfc_cnn_trainer* T) {
    if (!T) return;
    if (T->stream) (void)hipStreamSynchronize(T->stream);
    delete T;
}

static int cnn_fill_samples(CnnNet& N, const double* const* pm1, const double* const* p0,
                            const double* const* psi, const double* const* pp1,
                            double* const* out) {
    if (!pm1 || !p0 || !psi) return fail(MPFC_EINVAL, "phi^{n-1}, phi^n and psi^n are required");
    for (int s = 0; s < N.B; ++s) {
        if (!pm1[s] || !p0[s] || !psi[s] || (pp1 && !pp1[s]) || (out && !out[s]))
            return fail(MPFC_EINVAL, "NULL sample buffer");
        N.h_smp[s] = CnnSample{pm1[s], p0[s], psi[s], pp1 ? pp1[s] : nullptr,
                               out ? out[s] : nullptr};
    }
    return MPFC_OK;
}

int mpfc_cnn_train_step(mpfc_cnn_trainer* T, const double* const* d_phi_nm1,
                        const double* const* d_phi_n, const double* const* d_psi_n,
                        const double* const* d_phi_np1, int update, double* h_loss,
                        float* h_grad) {
    if (!T) return fail(MPFC_EINVAL, "trainer is NULL");
    if (!d_phi_np1) return fail(MPFC_EINVAL, "phi^{n+1} is required");
    CnnNet& N = T->net;
    int rc = cnn_fill_samples(N, d_phi_nm1, d_phi_n, d_psi_n, d_phi_np1, nullptr);
    if (!rc) rc = N.set_samples(T->stream);
    if (rc) return rc;
    N.forward(T->stream, true);
    N.backward(T->stream);
    HIP_TRY(hipMemcpyAsync(N.h_sums, N.sums, N.B * sizeof(double), hipMemcpyDeviceToHost, T->stream));
    if (h_grad)
        HIP_TRY(hipMemcpyAsync(h_grad, N.grad, CNN_NPARAM * sizeof(float), hipMemcpyDeviceToHost,
                               T->stream));
    if (update) N.adam(T->hp, T->stream);
    HIP_TRY(hipStreamSynchronize(T->stream));
    HIP_TRY(hipGetLastError());
    double loss = 0.0;
    for (int s = 0; s < N.B; ++s) loss += N.h_sums[s];
    if (h_loss) *h_loss = loss / ((double)N.B * (double)N.NP);
    if (!std::isfinite(loss)) return fail(MPFC_ENONFINITE, "training loss is not finite");
    return MPFC_OK;
}

int mpfc_cnn_predict(mpfc_cnn_trainer* T, const double* const* d_phi_nm1,
                     const double* const* d_phi_n, const double* const* d_psi_n,
                     double* const* d_guess) {
    if (!T) return fail(MPFC_EINVAL, "trainer is NULL");
    if (!d_guess) return fail(MPFC_EINVAL, "outputs are required");
    CnnNet& N = T->net;
    int rc = cnn_fill_samples(N, d_phi_nm1, d_phi_n, d_psi_n, nullptr, d_guess);
    if (!rc) rc = N.set_samples(T->stream);
    if (rc) return rc;
    N.forward(T->stream, false);
    HIP_TRY(hipStreamSynchronize(T->stream));
    HIP_TRY(hipGetLastError());
    return MPFC_OK;
}

int mpfc_cnn_trainer_set_lr(mpfc_cnn_trainer* T, float lr) {
    if (!T || !(lr > 0)) return fail(MPFC_EINVAL, "trainer is NULL or lr <= 0");
    T->hp.lr = lr;
    return MPFC_OK;
}

int mpfc_cnn_trainer_blob(mpfc_cnn_trainer* T, float* blob, size_t count) {
    if (!T || !blob) return fail(MPFC_EINVAL, "trainer and blob are required");
    if (count != (size_t)CNN_BLOB) return fail(MPFC_EINVAL, "blob has the wrong size");
    const float hdr[CNN_BLOB_HEADER] = {2.f, (float)CNN_CIN, (float)CNN_CH, 4.f,
                                        (float)T->net.in_scale, (float)T->net.out_scale,
                                        (float)T->net.dt, 0.f};
    std::memcpy(blob, hdr, sizeof hdr);
    HIP_TRY(hipMemcpyAsync(blob + CNN_BLOB_HEADER, T->net.theta, CNN_NPARAM * sizeof(float),
                           hipMemcpyDeviceToHost, T->stream));
    HIP_TRY(hipStreamSynchronize(T->stream));
    return MPFC_OK;
}

}  // extern "C"
