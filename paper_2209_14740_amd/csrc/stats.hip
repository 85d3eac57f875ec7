// Statistics of the stochastic Galerkin solution u_m(x, ξ) = Σ_i V_i(x) φ_i(ξ) (eq.
// Galerkin_approx), the post-processing of Section 7 (Figures bE_Var and k123_convergence):
//   E[u_m] = V_0,   Var[Re u_m] = Σ_{i>=1} (Re V_i)²,   Var[Im u_m] = Σ_{i>=1} (Im V_i)²
// (orthonormal basis with φ_0 = 1, so E[φ_i] = 0 and E[φ_i φ_j] = δ_ij for i, j >= 1), and
// the per-degree magnitudes γ_j = max{ ||V_i||_∞ : deg φ_i = j } (eq. magnitude_V).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "sg_internal.h"

namespace sgi {

namespace {

constexpr int ST = 256;

__global__ __launch_bounds__(ST) void k_moments(const double2* __restrict__ V, long long P, int Q,
                                                double2* __restrict__ mean, double* __restrict__ var) {
    for (long long p = (long long)blockIdx.x * ST + threadIdx.x; p < P; p += (long long)gridDim.x * ST) {
        double vr = 0.0, vi = 0.0;
        for (int q = 1; q < Q; ++q) {
            const double2 v = V[(long long)q * P + p];
            vr = fma(v.x, v.x, vr);
            vi = fma(v.y, v.y, vi);
        }
        if (mean) mean[p] = V[p];
        if (var) {
            var[p] = vr;
            var[P + p] = vi;
        }
    }
}

// partial[q][b] = max_{p in block b's share of plane q} |V_q(p)|
__global__ __launch_bounds__(ST) void k_plane_max(const double2* __restrict__ V, long long P, int nb,
                                                  double* __restrict__ partial) {
    __shared__ double red[ST / 64];
    const int q = blockIdx.y;
    double m = 0.0;
    for (long long p = (long long)blockIdx.x * ST + threadIdx.x; p < P; p += (long long)nb * ST) {
        const double2 v = V[(long long)q * P + p];
        m = fmax(m, hypot(v.x, v.y));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = red[0];
        for (int w = 1; w < ST / 64; ++w) t = fmax(t, red[w]);
        partial[(long long)q * nb + blockIdx.x] = t;
    }
}

}  // namespace

int launch_moments(const Ctx* c, const double2* x, double2* mean, double* var, hipStream_t st) {
    const long long P = c->P;
    long long blocks = (P + ST - 1) / ST;
    blocks = std::max(1LL, std::min(blocks, 4096LL));
    KScope ks(SG_K_AXPY, 16.0 * (double)c->Q * P + 32.0 * P, st);
    hipLaunchKernelGGL(k_moments, dim3((unsigned)blocks), dim3(ST), 0, st, x, P, c->Q, mean, var);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int degree_magnitudes(const Ctx* c, const double2* x, double* gamma, hipStream_t st) {
    const long long P = c->P;
    const int nb = (int)std::max(1LL, std::min((P + ST - 1) / ST, 256LL));
    double* d = nullptr;
    SG_HIP(hipMalloc(&d, (size_t)nb * c->Q * sizeof(double)));
    hipLaunchKernelGGL(k_plane_max, dim3(nb, c->Q), dim3(ST), 0, st, x, P, nb, d);
    hipError_t e = hipGetLastError();
    std::vector<double> h((size_t)nb * c->Q);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, h.size() * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    SG_HIP(e);
    for (int j = 0; j <= c->degree; ++j) gamma[j] = 0.0;
    for (int q = 0; q < c->Q; ++q) {
        int deg = 0;
        for (int l = 0; l < c->s; ++l) deg += c->alpha[(size_t)q * c->s + l];
        double m = 0.0;
        for (int b = 0; b < nb; ++b) m = std::max(m, h[(size_t)q * nb + b]);
        if (!std::isfinite(m)) return fail(SG_ENONFINITE, "non-finite coefficient");
        gamma[deg] = std::max(gamma[deg], m);
    }
    return SG_OK;
}

}  // namespace sgi
