// Internal declarations of the learned correction network (net.hip kernels, net_host.cpp host).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sg_internal.h"

namespace sgi {

// net.hip launchers (BF16 tensors are uint16_t bit patterns)
int net_conv(const uint16_t* X, int Cin, const uint16_t* W, const float* bias, void* Y, int Cout, bool relu, bool out_f32,
             const uint16_t* mask, int H, int Wd, int batch, int ks, hipStream_t st);
long long net_wgrad_scratch(int Cout, int Cin, int ks, int H, int Wd, int batch);
long long net_colsum_scratch(int Cout, int H, int Wd, int batch);
int net_wgrad(const uint16_t* dZ, int Cout, const uint16_t* X, int Cin, int H, int Wd, int batch, int ks, int co_real,
              int ci_real, float* scratch, float* gW, float* gb, float* scratch_b, hipStream_t st);
int net_pool(const uint16_t* in, uint16_t* out, int Hl, int Wl, int C, int batch, hipStream_t st);
int net_up_concat(const uint16_t* U, int Cu, const uint16_t* S, int Cs, uint16_t* out, int H, int Wd, int batch,
                  hipStream_t st);
int net_up_bwd(const uint16_t* dC, int C, int Cu, const uint16_t* mask, uint16_t* out, int Hl, int Wl, int batch,
               hipStream_t st);
int net_skip_bwd(const uint16_t* dC, int Ccat, int Cu, const uint16_t* dP, const uint16_t* mask, uint16_t* out, int H,
                 int Wd, int C, int batch, hipStream_t st);
int net_pack(const double2* r, const double2* rnorm, int Q, int n, int H, const double* kf, int s, double kbar, int Cp,
             uint16_t* out, hipStream_t st);
int net_unpack_add(const float* y, int Cp, const double2* znorm, int Q, int n, int H, double2* z, hipStream_t st);
int net_pack_target(const double2* c, const double2* znorm, int Q, int n, int H, int Cp, float* out, hipStream_t st);
int net_to_bf16(const float* in, int C, uint16_t* out, int Cp, long long npix, hipStream_t st);
int net_pad_f32(const float* in, int C, float* out, int Cp, long long npix, hipStream_t st);
int net_unpad_f32(const float* in, int Cp, float* out, int C, long long npix, hipStream_t st);
int net_mse(const float* y, const float* t, long long npix, int Cp, int C, double inv_count, uint16_t* dy, float* partial,
            int nblocks, hipStream_t st);
int net_adam(float* th, float* m, float* v, const float* g, long long n, float lr, float b1, float b2, float eps, int t,
             hipStream_t st);
int net_weights(const float* th, int co_real, int ci_real, int ks, int Coutp, int Cinp, uint16_t* wf, uint16_t* wb,
                float* bias, hipStream_t st);

struct NetLayer {
    int ks, ci, co, cip, cop;       // kernel size, real and padded channel counts
    long long off;                  // offset of W in the flat parameters (bias follows)
    uint16_t* wf = nullptr;         // [cop][ks²][cip]
    uint16_t* wb = nullptr;         // [cip][ks²][cop], taps reversed
    float* bias = nullptr;          // [cop]
};

// 3-level U-Net (widths 32, 64, 128) of the learned preconditioner.
struct Net {
    int Q = 0, s = 0, cin = 0, cout = 0, cinp = 0, coutp = 0;
    int device = 0;
    long long nparams = 0;
    std::vector<NetLayer> L;
    float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    int adam_t = 0;
    // activations / gradients, sized for (cap_batch, cap_H)
    int cap_batch = 0, cap_H = 0;
    std::vector<void*> bufs;
    uint16_t *x = nullptr, *e0a = nullptr, *s0 = nullptr, *p0 = nullptr, *e1a = nullptr, *s1 = nullptr, *p1 = nullptr,
             *ba = nullptr, *bt = nullptr, *c1 = nullptr, *d1a = nullptr, *d1 = nullptr, *c0 = nullptr, *d0a = nullptr,
             *d0 = nullptr;
    float *y = nullptr, *tgt = nullptr;
    uint16_t *dy = nullptr, *gL0a = nullptr, *gL0b = nullptr, *gc0 = nullptr, *gL1a = nullptr, *gL1b = nullptr,
             *gc1 = nullptr, *gL2a = nullptr, *gL2b = nullptr, *gp1 = nullptr, *gp0 = nullptr;
    float *wscratch = nullptr, *bscratch = nullptr, *lpartial = nullptr, *fbuf = nullptr;
    int lblocks = 0;
    // preconditioner scratch
    double2* nrm = nullptr;         // device norms: [0] ||v||, [1] ||A_0^{-1} v||, per sample in training
    int nrm_cap = 0;
    double2* npartial = nullptr;
    long long npartial_cap = 0;
    double2* vtmp = nullptr;        // training: A_0^{-1} r and the correction
    long long vtmp_cap = 0;
    float* hpinned = nullptr;
    int hpinned_cap = 0;
    ~Net();
};

int net_create(int Q, int s, unsigned long long seed, Net** out);
int net_set_params(Net* n, const float* host);
int net_get_params(Net* n, float* host);
int net_forward(Net* n, int batch, int H, hipStream_t st);
int net_backward(Net* n, int batch, int H, double* loss, hipStream_t st);
int net_forward_nhwc(Net* n, int batch, int H, const float* x, float* y, hipStream_t st);
int net_grad_nhwc(Net* n, int batch, int H, const float* x, const float* t, double* loss, float* grad_host,
                  hipStream_t st);
int net_adam_step(Net* n, float lr, hipStream_t st);
int net_train_pairs(Net* n, int batch, Ctx* const* c, const double2* const* r, const double2* const* e, float lr,
                    int precision, double* loss, hipStream_t st);
int net_precond(Net* n, Ctx* c, int precision, const double2* v, double2* z, hipStream_t st);
int net_save(Net* n, const char* path);
int net_load(Net* n, const char* path);

}  // namespace sgi
