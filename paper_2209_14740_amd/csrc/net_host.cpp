// Host side of the learned correction network: parameters, buffers, the forward and
// backward sequences of the U-Net, Adam, training on (residual, error) pairs, and the
// learned preconditioner z = A_0^{-1} v + ||A_0^{-1} v|| / sqrt(Q n²) · N(v; k fields).
//
// Network (widths 32, 64, 128; every 3×3 convolution is followed by ReLU):
//   s0 = conv(conv(x))                         level 0 (H × H)
//   s1 = conv(conv(pool s0))                   level 1 (H/2)
//   bt = conv(conv(pool s1))                   level 2 (H/4)
//   d1 = conv(conv([up bt, s1]))               level 1
//   d0 = conv(conv([up d1, s0]))               level 0
//   y  = head(d0)                              1×1, linear, FP32 output
// Flat parameters: per layer W[co][kh][kw][ci] then b[co], layers in the order above.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <vector>

#include "net_internal.h"

namespace sgi {

namespace {

constexpr int W0 = 32, W1 = 64, W2 = 128;
inline int pad32(int c) { return (c + 31) / 32 * 32; }

// SplitMix64 (Steele, Lea & Flood, 2014): counter-based 64-bit generator.
inline uint64_t splitmix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
inline double uniform01(uint64_t seed, uint64_t i) {
    return ((splitmix64(seed ^ splitmix64(i)) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

enum { ENC0A, ENC0B, ENC1A, ENC1B, BOTA, BOTB, DEC1A, DEC1B, DEC0A, DEC0B, HEAD, NLAYER };

int refresh_weights(Net* n, hipStream_t st) {
    for (auto& l : n->L) {
        int rc = net_weights(n->theta + l.off, l.co, l.ci, l.ks, l.cop, l.cip, l.wf, l.wb, l.bias, st);
        if (rc) return rc;
    }
    return SG_OK;
}

template <class T>
int nalloc(Net* n, T** p, size_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, count * sizeof(T) + 256) != hipSuccess) return fail(SG_ENOMEM, "network buffer allocation failed");
    n->bufs.push_back(q);
    *p = reinterpret_cast<T*>(q);
    return SG_OK;
}

int ensure_buffers(Net* n, int batch, int H) {
    if (H < 4 || H % 4) return fail(SG_EINVAL, "network image size must be a positive multiple of 4");
    if (batch < 1) return fail(SG_EINVAL, "batch must be >= 1");
    if (n->cap_batch >= batch && n->cap_H == H) return SG_OK;
    for (void* p : n->bufs) (void)hipFree(p);
    n->bufs.clear();
    n->cap_batch = n->cap_H = 0;
    const size_t B = batch, P0 = (size_t)H * H, P1 = P0 / 4, P2 = P0 / 16;
    int rc = 0;
    auto A = [&](uint16_t** p, size_t cnt) { if (!rc) rc = nalloc(n, p, cnt); };
    auto F = [&](float** p, size_t cnt) { if (!rc) rc = nalloc(n, p, cnt); };
    A(&n->x, B * P0 * n->cinp);
    A(&n->e0a, B * P0 * W0);
    A(&n->s0, B * P0 * W0);
    A(&n->p0, B * P1 * W0);
    A(&n->e1a, B * P1 * W1);
    A(&n->s1, B * P1 * W1);
    A(&n->p1, B * P2 * W1);
    A(&n->ba, B * P2 * W2);
    A(&n->bt, B * P2 * W2);
    A(&n->c1, B * P1 * (W2 + W1));
    A(&n->d1a, B * P1 * W1);
    A(&n->d1, B * P1 * W1);
    A(&n->c0, B * P0 * (W1 + W0));
    A(&n->d0a, B * P0 * W0);
    A(&n->d0, B * P0 * W0);
    F(&n->y, B * P0 * n->coutp);
    F(&n->tgt, B * P0 * n->coutp);
    A(&n->dy, B * P0 * n->coutp);
    A(&n->gL0a, B * P0 * W0);
    A(&n->gL0b, B * P0 * W0);
    A(&n->gc0, B * P0 * (W1 + W0));
    A(&n->gL1a, B * P1 * W1);
    A(&n->gL1b, B * P1 * W1);
    A(&n->gc1, B * P1 * (W2 + W1));
    A(&n->gL2a, B * P2 * W2);
    A(&n->gL2b, B * P2 * W2);
    A(&n->gp1, B * P2 * W1);
    A(&n->gp0, B * P1 * W0);
    long long ws = 0, bs = 0;
    for (int i = 0; i < NLAYER; ++i) {
        const NetLayer& l = n->L[i];
        const int lev = (i == BOTA || i == BOTB) ? 2 : (i == ENC1A || i == ENC1B || i == DEC1A || i == DEC1B) ? 1 : 0;
        const int h = H >> lev;
        ws = std::max(ws, net_wgrad_scratch(l.cop, l.cip, l.ks, h, h, batch));
        bs = std::max(bs, net_colsum_scratch(l.cop, h, h, batch));
    }
    F(&n->wscratch, (size_t)ws);
    F(&n->bscratch, (size_t)bs);
    n->lblocks = 1024;
    F(&n->lpartial, (size_t)n->lblocks);
    F(&n->fbuf, B * P0 * std::max(n->cinp, n->coutp));
    if (rc) return rc;
    n->cap_batch = batch;
    n->cap_H = H;
    return SG_OK;
}

int ensure_pinned(Net* n, int count) {
    if (n->hpinned_cap >= count) return SG_OK;
    if (n->hpinned) (void)hipHostFree(n->hpinned);
    n->hpinned = nullptr;
    n->hpinned_cap = 0;
    SG_HIP(hipHostMalloc(&n->hpinned, (size_t)count * sizeof(float), hipHostMallocDefault));
    n->hpinned_cap = count;
    return SG_OK;
}

// ||x|| of an SG vector into the device scalar out (two-stage deterministic reduction)
int dev_norm(Net* n, long long len, const double2* x, double2* out, hipStream_t st) {
    const int nb = reduction_blocks(len);
    if (n->npartial_cap < nb) {
        if (n->npartial) (void)hipFree(n->npartial);
        n->npartial = nullptr;
        n->npartial_cap = 0;
        if (hipMalloc(&n->npartial, (size_t)nb * sizeof(double2)) != hipSuccess)
            return fail(SG_ENOMEM, "network norm scratch allocation failed");
        n->npartial_cap = nb;
    }
    int rc = launch_norm2(len, x, n->npartial, nb, st);
    if (rc) return rc;
    return launch_reduce_norm(nb, n->npartial, out, st);
}

int ensure_norms(Net* n, int count) {
    if (n->nrm_cap >= count) return SG_OK;
    if (n->nrm) (void)hipFree(n->nrm);
    n->nrm = nullptr;
    n->nrm_cap = 0;
    if (hipMalloc(&n->nrm, (size_t)count * sizeof(double2)) != hipSuccess)
        return fail(SG_ENOMEM, "network scalar allocation failed");
    n->nrm_cap = count;
    return SG_OK;
}

}  // namespace

Net::~Net() {
    for (void* p : bufs) (void)hipFree(p);
    for (auto& l : L) {
        (void)hipFree(l.wf);
        (void)hipFree(l.wb);
        (void)hipFree(l.bias);
    }
    (void)hipFree(theta);
    (void)hipFree(m);
    (void)hipFree(v);
    (void)hipFree(grad);
    (void)hipFree(nrm);
    (void)hipFree(npartial);
    (void)hipFree(vtmp);
    if (hpinned) (void)hipHostFree(hpinned);
}

int net_create(int Q, int s, unsigned long long seed, Net** out) {
    if (Q < 1 || s < 0 || 2 * Q + s + 1 > 256 || 2 * Q > 256) return fail(SG_EINVAL, "network: unsupported Q or s");
    Net* n = new Net();
    std::unique_ptr<Net> guard(n);
    SG_HIP(hipGetDevice(&n->device));
    n->Q = Q;
    n->s = s;
    n->cin = 2 * Q + s + 1;
    n->cout = 2 * Q;
    n->cinp = pad32(n->cin);
    n->coutp = pad32(n->cout);
    const int spec[NLAYER][3] = {{3, n->cin, W0}, {3, W0, W0},      {3, W0, W1},      {3, W1, W1},
                                 {3, W1, W2},     {3, W2, W2},      {3, W2 + W1, W1}, {3, W1, W1},
                                 {3, W1 + W0, W0}, {3, W0, W0},     {1, W0, n->cout}};
    long long off = 0;
    for (int i = 0; i < NLAYER; ++i) {
        NetLayer l;
        l.ks = spec[i][0];
        l.ci = spec[i][1];
        l.co = spec[i][2];
        l.cip = pad32(l.ci);
        l.cop = pad32(l.co);
        l.off = off;
        off += (long long)l.co * l.ks * l.ks * l.ci + l.co;
        const size_t nw = (size_t)l.cop * l.ks * l.ks * l.cip;
        n->L.push_back(l);
        NetLayer& ll = n->L.back();   // owned by n from here on
        if (hipMalloc(&ll.wf, nw * 2) != hipSuccess || hipMalloc(&ll.wb, nw * 2) != hipSuccess ||
            hipMalloc(&ll.bias, (size_t)l.cop * 4) != hipSuccess)
            return fail(SG_ENOMEM, "network weight allocation failed");
    }
    n->nparams = off;
    const size_t bytes = (size_t)off * sizeof(float);
    if (hipMalloc(&n->theta, bytes) != hipSuccess || hipMalloc(&n->m, bytes) != hipSuccess ||
        hipMalloc(&n->v, bytes) != hipSuccess || hipMalloc(&n->grad, bytes) != hipSuccess)
        return fail(SG_ENOMEM, "network parameter allocation failed");
    // He-normal initialisation (std sqrt(2/fan_in), head ×0.1), zero biases
    std::vector<float> th((size_t)off, 0.f);
    uint64_t ctr = 0;
    for (int i = 0; i < NLAYER; ++i) {
        const NetLayer& l = n->L[i];
        const double sd = std::sqrt(2.0 / (l.ks * l.ks * l.ci)) * (i == HEAD ? 0.1 : 1.0);
        const long long nw = (long long)l.co * l.ks * l.ks * l.ci;
        for (long long k = 0; k < nw; ++k, ctr += 2) {
            const double u1 = uniform01(seed, ctr), u2 = uniform01(seed, ctr + 1);
            th[l.off + k] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
        }
    }
    int rc = net_set_params(n, th.data());
    if (rc) return rc;
    *out = guard.release();
    return SG_OK;
}

int net_set_params(Net* n, const float* host) {
    const size_t bytes = (size_t)n->nparams * sizeof(float);
    SG_HIP(hipMemcpy(n->theta, host, bytes, hipMemcpyHostToDevice));
    SG_HIP(hipMemset(n->m, 0, bytes));
    SG_HIP(hipMemset(n->v, 0, bytes));
    SG_HIP(hipMemset(n->grad, 0, bytes));
    n->adam_t = 0;
    int rc = refresh_weights(n, nullptr);
    if (rc) return rc;
    SG_HIP(hipDeviceSynchronize());
    return SG_OK;
}

int net_get_params(Net* n, float* host) {
    SG_HIP(hipDeviceSynchronize());
    SG_HIP(hipMemcpy(host, n->theta, (size_t)n->nparams * sizeof(float), hipMemcpyDeviceToHost));
    return SG_OK;
}

// Forward pass of the whole network on n->x → n->y (FP32, coutp channels).
int net_forward(Net* n, int B, int H, hipStream_t st) {
    int rc = ensure_buffers(n, B, H);
    if (rc) return rc;
    const int H1 = H / 2, H2 = H / 4;
    const auto& L = n->L;
    auto conv = [&](int li, const uint16_t* in, void* out, int h, bool relu) {
        const NetLayer& l = L[li];
        return net_conv(in, l.cip, l.wf, l.bias, out, l.cop, relu, li == HEAD, nullptr, h, h, B, l.ks, st);
    };
    if ((rc = conv(ENC0A, n->x, n->e0a, H, true))) return rc;
    if ((rc = conv(ENC0B, n->e0a, n->s0, H, true))) return rc;
    if ((rc = net_pool(n->s0, n->p0, H1, H1, W0, B, st))) return rc;
    if ((rc = conv(ENC1A, n->p0, n->e1a, H1, true))) return rc;
    if ((rc = conv(ENC1B, n->e1a, n->s1, H1, true))) return rc;
    if ((rc = net_pool(n->s1, n->p1, H2, H2, W1, B, st))) return rc;
    if ((rc = conv(BOTA, n->p1, n->ba, H2, true))) return rc;
    if ((rc = conv(BOTB, n->ba, n->bt, H2, true))) return rc;
    if ((rc = net_up_concat(n->bt, W2, n->s1, W1, n->c1, H1, H1, B, st))) return rc;
    if ((rc = conv(DEC1A, n->c1, n->d1a, H1, true))) return rc;
    if ((rc = conv(DEC1B, n->d1a, n->d1, H1, true))) return rc;
    if ((rc = net_up_concat(n->d1, W1, n->s0, W0, n->c0, H, H, B, st))) return rc;
    if ((rc = conv(DEC0A, n->c0, n->d0a, H, true))) return rc;
    if ((rc = conv(DEC0B, n->d0a, n->d0, H, true))) return rc;
    return conv(HEAD, n->d0, n->y, H, false);
}

// Loss against n->tgt and the gradient of the mean loss into n->grad (flat FP32).
// The loss value is copied back only if loss != NULL (that synchronises the stream).
int net_backward(Net* n, int B, int H, double* loss, hipStream_t st) {
    const int H1 = H / 2, H2 = H / 4;
    const long long npix = (long long)B * H * H;
    const auto& L = n->L;
    int rc = net_mse(n->y, n->tgt, npix, n->coutp, n->cout, 1.0 / ((double)npix * n->cout), n->dy, n->lpartial,
                     n->lblocks, st);
    if (rc) return rc;
    // weight gradient of layer li from dZ (its pre-activation gradient) and its input X
    auto wg = [&](int li, const uint16_t* dZ, const uint16_t* X, int h) {
        const NetLayer& l = L[li];
        float* g = n->grad + l.off;
        return net_wgrad(dZ, l.cop, X, l.cip, h, h, B, l.ks, l.co, l.ci, n->wscratch, g,
                         g + (long long)l.co * l.ks * l.ks * l.ci, n->bscratch, st);
    };
    // input gradient of layer li (transposed, tap-flipped weights), optionally times a ReLU mask
    auto dg = [&](int li, const uint16_t* dZ, uint16_t* out, const uint16_t* mask, int h) {
        const NetLayer& l = L[li];
        return net_conv(dZ, l.cop, l.wb, nullptr, out, l.cip, false, false, mask, h, h, B, l.ks, st);
    };
    if ((rc = wg(HEAD, n->dy, n->d0, H))) return rc;
    if ((rc = dg(HEAD, n->dy, n->gL0a, n->d0, H))) return rc;
    if ((rc = wg(DEC0B, n->gL0a, n->d0a, H))) return rc;
    if ((rc = dg(DEC0B, n->gL0a, n->gL0b, n->d0a, H))) return rc;
    if ((rc = wg(DEC0A, n->gL0b, n->c0, H))) return rc;
    if ((rc = dg(DEC0A, n->gL0b, n->gc0, nullptr, H))) return rc;
    if ((rc = net_up_bwd(n->gc0, W1 + W0, W1, n->d1, n->gL1a, H1, H1, B, st))) return rc;
    if ((rc = wg(DEC1B, n->gL1a, n->d1a, H1))) return rc;
    if ((rc = dg(DEC1B, n->gL1a, n->gL1b, n->d1a, H1))) return rc;
    if ((rc = wg(DEC1A, n->gL1b, n->c1, H1))) return rc;
    if ((rc = dg(DEC1A, n->gL1b, n->gc1, nullptr, H1))) return rc;
    if ((rc = net_up_bwd(n->gc1, W2 + W1, W2, n->bt, n->gL2a, H2, H2, B, st))) return rc;
    if ((rc = wg(BOTB, n->gL2a, n->ba, H2))) return rc;
    if ((rc = dg(BOTB, n->gL2a, n->gL2b, n->ba, H2))) return rc;
    if ((rc = wg(BOTA, n->gL2b, n->p1, H2))) return rc;
    if ((rc = dg(BOTA, n->gL2b, n->gp1, nullptr, H2))) return rc;
    if ((rc = net_skip_bwd(n->gc1, W2 + W1, W2, n->gp1, n->s1, n->gL1a, H1, H1, W1, B, st))) return rc;
    if ((rc = wg(ENC1B, n->gL1a, n->e1a, H1))) return rc;
    if ((rc = dg(ENC1B, n->gL1a, n->gL1b, n->e1a, H1))) return rc;
    if ((rc = wg(ENC1A, n->gL1b, n->p0, H1))) return rc;
    if ((rc = dg(ENC1A, n->gL1b, n->gp0, nullptr, H1))) return rc;
    if ((rc = net_skip_bwd(n->gc0, W1 + W0, W1, n->gp0, n->s0, n->gL0a, H, H, W0, B, st))) return rc;
    if ((rc = wg(ENC0B, n->gL0a, n->e0a, H))) return rc;
    if ((rc = dg(ENC0B, n->gL0a, n->gL0b, n->e0a, H))) return rc;
    if ((rc = wg(ENC0A, n->gL0b, n->x, H))) return rc;
    if (loss) {
        if ((rc = ensure_pinned(n, n->lblocks))) return rc;
        SG_HIP(hipMemcpyAsync(n->hpinned, n->lpartial, (size_t)n->lblocks * sizeof(float), hipMemcpyDeviceToHost, st));
        SG_HIP(hipStreamSynchronize(st));
        double s = 0;
        for (int i = 0; i < n->lblocks; ++i) s += n->hpinned[i];
        *loss = s / ((double)npix * n->cout);
    }
    return SG_OK;
}

int net_forward_nhwc(Net* n, int B, int H, const float* x, float* y, hipStream_t st) {
    int rc = ensure_buffers(n, B, H);
    if (rc) return rc;
    const long long npix = (long long)B * H * H;
    if ((rc = net_to_bf16(x, n->cin, n->x, n->cinp, npix, st))) return rc;
    if ((rc = net_forward(n, B, H, st))) return rc;
    return net_unpad_f32(n->y, n->coutp, y, n->cout, npix, st);
}

int net_grad_nhwc(Net* n, int B, int H, const float* x, const float* t, double* loss, float* grad_host, hipStream_t st) {
    int rc = ensure_buffers(n, B, H);
    if (rc) return rc;
    const long long npix = (long long)B * H * H;
    if ((rc = net_to_bf16(x, n->cin, n->x, n->cinp, npix, st))) return rc;
    if ((rc = net_pad_f32(t, n->cout, n->tgt, n->coutp, npix, st))) return rc;
    if ((rc = net_forward(n, B, H, st))) return rc;
    double l = 0;
    if ((rc = net_backward(n, B, H, &l, st))) return rc;
    if (loss) *loss = l;
    if (grad_host) {
        SG_HIP(hipMemcpyAsync(grad_host, n->grad, (size_t)n->nparams * sizeof(float), hipMemcpyDeviceToHost, st));
        SG_HIP(hipStreamSynchronize(st));
    }
    return SG_OK;
}

int net_adam_step(Net* n, float lr, hipStream_t st) {
    n->adam_t += 1;
    int rc = net_adam(n->theta, n->m, n->v, n->grad, n->nparams, lr, 0.9f, 0.999f, 1e-8f, n->adam_t, st);
    if (rc) return rc;
    return refresh_weights(n, st);
}

static int check_ctx(Net* n, Ctx* c) {
    if (c->dim != 2) return fail(SG_EINVAL, "the learned preconditioner needs a 2D problem");
    if (c->Q != n->Q || c->s != n->s) return fail(SG_EINVAL, "network was built for another Q or s");
    return SG_OK;
}

int net_train_pairs(Net* n, int B, Ctx* const* cs, const double2* const* r, const double2* const* e, float lr,
                    int precision, double* loss, hipStream_t st) {
    if (B < 1 || !cs || !r || !e) return fail(SG_EINVAL, "invalid training batch");
    const int nn = cs[0]->n, H = (nn + 3) / 4 * 4;
    for (int i = 0; i < B; ++i) {
        if (!cs[i] || !r[i] || !e[i]) return fail(SG_EINVAL, "null entry in the training batch");
        int rc = check_ctx(n, cs[i]);
        if (rc) return rc;
        if (cs[i]->n != nn) return fail(SG_EINVAL, "a training batch must share one grid size");
    }
    int rc = ensure_buffers(n, B, H);
    if (rc) return rc;
    if ((rc = ensure_norms(n, 2 * B))) return rc;
    const long long len = cs[0]->nvec;
    if (n->vtmp_cap < len) {
        if (n->vtmp) (void)hipFree(n->vtmp);
        n->vtmp = nullptr;
        n->vtmp_cap = 0;
        if (hipMalloc(&n->vtmp, (size_t)len * sizeof(double2)) != hipSuccess)
            return fail(SG_ENOMEM, "training scratch allocation failed");
        n->vtmp_cap = len;
    }
    const long long P = (long long)H * H;
    for (int i = 0; i < B; ++i) {
        Ctx* c = cs[i];
        // target correction e - A_0^{-1} r in units of ||A_0^{-1} r|| / sqrt(Q n²)
        if ((rc = launch_precond(c, SG_PC_MEAN, precision, r[i], n->vtmp, st))) return rc;
        if ((rc = dev_norm(n, len, r[i], n->nrm + 2 * i, st))) return rc;
        if ((rc = dev_norm(n, len, n->vtmp, n->nrm + 2 * i + 1, st))) return rc;
        if ((rc = launch_axpby(len, make_double2(1, 0), e[i], make_double2(-1, 0), n->vtmp, n->vtmp, st))) return rc;
        if ((rc = net_pack(r[i], n->nrm + 2 * i, c->Q, c->n, H, c->d_kf, c->s, c->kbar, n->cinp, n->x + i * P * n->cinp,
                           st)))
            return rc;
        if ((rc = net_pack_target(n->vtmp, n->nrm + 2 * i + 1, c->Q, c->n, H, n->coutp, n->tgt + i * P * n->coutp, st)))
            return rc;
    }
    if ((rc = net_forward(n, B, H, st))) return rc;
    if ((rc = net_backward(n, B, H, loss, st))) return rc;
    return net_adam_step(n, lr, st);
}

int net_precond(Net* n, Ctx* c, int precision, const double2* v, double2* z, hipStream_t st) {
    int rc = check_ctx(n, c);
    if (rc) return rc;
    if (v == z) return fail(SG_EINVAL, "the learned preconditioner needs distinct input and output");
    const int H = (c->n + 3) / 4 * 4;
    if ((rc = ensure_buffers(n, 1, H))) return rc;
    if ((rc = ensure_norms(n, 2))) return rc;
    if ((rc = launch_precond(c, SG_PC_MEAN, precision, v, z, st))) return rc;
    if ((rc = dev_norm(n, c->nvec, v, n->nrm, st))) return rc;
    if ((rc = dev_norm(n, c->nvec, z, n->nrm + 1, st))) return rc;
    if ((rc = net_pack(v, n->nrm, c->Q, c->n, H, c->d_kf, c->s, c->kbar, n->cinp, n->x, st))) return rc;
    if ((rc = net_forward(n, 1, H, st))) return rc;
    return net_unpack_add(n->y, n->coutp, n->nrm + 1, c->Q, c->n, H, z, st);
}

int net_save(Net* n, const char* path) {
    std::vector<float> th((size_t)n->nparams);
    int rc = net_get_params(n, th.data());
    if (rc) return rc;
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(SG_EINVAL, std::string("cannot open ") + path);
    const char magic[8] = {'S', 'G', 'U', 'N', 'E', 'T', '1', 0};
    const long long hdr[3] = {n->Q, n->s, n->nparams};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(long long), 3, f) == 3 &&
              std::fwrite(th.data(), sizeof(float), th.size(), f) == th.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? SG_OK : fail(SG_EINVAL, std::string("write failed: ") + path);
}

int net_load(Net* n, const char* path) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(SG_EINVAL, std::string("cannot open ") + path);
    char magic[8];
    long long hdr[3];
    std::vector<float> th((size_t)n->nparams);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "SGUNET1", 8) == 0 &&
              std::fread(hdr, sizeof(long long), 3, f) == 3 && hdr[0] == n->Q && hdr[1] == n->s &&
              hdr[2] == n->nparams && std::fread(th.data(), sizeof(float), th.size(), f) == th.size();
    std::fclose(f);
    if (!ok) return fail(SG_EINVAL, std::string("not a network file of this shape: ") + path);
    return net_set_params(n, th.data());
}

}  // namespace sgi
