// Matrix-free SG operator y = A x (Theorem 3.3, Theorems A.2 / A.4, eqs. b_ij / c_ij):
//
//   y_i(p) = (L x_i)(p) - Σ_j c_ij(p) x_j(p) - i Σ_j b_ij(p) x_j(p),
//   c_ij(p) = Σ_γ D2_γ(p) G_γ[i,j],   b_ij(p) = Σ_γ D1_γ(p) G_γ[i,j]   (boundary only),
//   (L u)(x_i, y_j) = d_j (T_x u) + d_i (T_y u),  T the 1D absorbing Laplacian of Theorem A.2.
//
// One workgroup owns a 64-point segment of one grid row and all Q coefficient blocks.
// The segment (with a one-point halo in x) and its coefficient fields are staged in LDS
// with coalesced 1 KB row loads; the four waves split the Q output blocks, each lane
// owning one grid point, so the coupling is lane-local and only the stencil reads the
// neighbours (x from LDS, y from global / L2).  The workgroup → row mapping keeps
// consecutive rows on one XCD so that the y-neighbour rows are L2 hits.
#include <hip/hip_runtime.h>

#include "apply_args.h"

namespace sgi {

namespace {

constexpr int TILE = 64;
constexpr int TPAD = TILE + 2;



__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ void apply_tile(const ApplyArgs& a, int tile, double2* smem) {
    double2* vt = smem;                                   // [Q][TPAD]
    double* dt = reinterpret_cast<double*>(smem + (size_t)a.Q * TPAD);   // [ng2][TILE]
    const int row = tile / a.ntiles_x;
    const int x0 = (tile % a.ntiles_x) * TILE;
    const int n = a.n;
    const long long P = a.P;
    const long long rowoff = (long long)row * n;

    for (int idx = threadIdx.x; idx < a.Q * TPAD; idx += blockDim.x) {
        const int q = idx / TPAD, l = idx - q * TPAD;
        const int xi = x0 + l - 1;
        double2 v = make_double2(0.0, 0.0);
        if (xi >= 0 && xi < n) v = a.x[(long long)q * P + rowoff + xi];
        vt[idx] = v;
    }
    for (int idx = threadIdx.x; idx < a.ng2 * TILE; idx += blockDim.x) {
        const int g = idx / TILE, l = idx - g * TILE;
        const int xi = x0 + l;
        dt[idx] = (xi < n) ? a.D2[(long long)g * P + rowoff + xi] : 0.0;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wv = uniform(threadIdx.x >> 6);
    const int xi = x0 + lane;
    if (xi >= n) return;
    const long long p = rowoff + xi;
    const bool is2d = a.dim == 2;
    const bool xb = (xi == 0 || xi == n - 1);
    const bool yb = is2d && (row == 0 || row == n - 1);
    const bool bnd = xb || yb;
    const double dx = xb ? 0.5 : 1.0;            // d_i
    const double dy = is2d ? (yb ? 0.5 : 1.0) : 1.0;   // d_j
    const int* prog = a.prog;
    const double* kv = a.vals + a.kv;

    for (int i = wv; i < a.Q; i += 4) {
        double re = 0.0, im = 0.0;
        const int pb = uniform(prog[a.kpp + i]), pe = uniform(prog[a.kpp + i + 1]);
        for (int pp = pb; pp < pe; ++pp) {
            const int j = uniform(prog[a.kpj + pp]);
            const int tb = uniform(prog[a.ktp + pp]), te = uniform(prog[a.ktp + pp + 1]);
            double cij = 0.0;
            for (int t = tb; t < te; ++t) cij += dt[prog[a.ktf + t] * TILE + lane] * kv[t];
            const double2 v = vt[j * TPAD + lane + 1];
            re += cij * v.x;
            im += cij * v.y;
        }
        // Laplacian: d_j (T_x u) + d_i (T_y u)
        const double2 uc = vt[i * TPAD + lane + 1];
        double2 tx;
        if (xi == 0) {
            const double2 ur = vt[i * TPAD + lane + 2];
            tx = make_double2(uc.x - ur.x, uc.y - ur.y);
        } else if (xi == n - 1) {
            const double2 ul = vt[i * TPAD + lane];
            tx = make_double2(uc.x - ul.x, uc.y - ul.y);
        } else {
            const double2 ul = vt[i * TPAD + lane], ur = vt[i * TPAD + lane + 2];
            tx = make_double2(2.0 * uc.x - ul.x - ur.x, 2.0 * uc.y - ul.y - ur.y);
        }
        double lre = dy * tx.x, lim = dy * tx.y;
        if (is2d) {
            const double2* xb_ = a.x + (long long)i * P;
            double2 ty;
            if (row == 0) {
                const double2 un = xb_[p + n];
                ty = make_double2(uc.x - un.x, uc.y - un.y);
            } else if (row == n - 1) {
                const double2 us = xb_[p - n];
                ty = make_double2(uc.x - us.x, uc.y - us.y);
            } else {
                const double2 us = xb_[p - n], un = xb_[p + n];
                ty = make_double2(2.0 * uc.x - us.x - un.x, 2.0 * uc.y - us.y - un.y);
            }
            lre += dx * ty.x;
            lim += dx * ty.y;
        }
        if (a.csl_beta != 0.0) {   // (1 + iβ) K x
            const double sre = re - a.csl_beta * im, sim = im + a.csl_beta * re;
            re = sre;
            im = sim;
        }
        double ore = lre * a.ih2 - re, oim = lim * a.ih2 - im;
        if (bnd) {
            // - i Σ_j b_ij x_j
            const double* bvv = a.vals + a.bv;
            const int qb = prog[a.bpp + i], qe = prog[a.bpp + i + 1];
            for (int pp = qb; pp < qe; ++pp) {
                const int j = prog[a.bpj + pp];
                double bij = 0.0;
                for (int t = prog[a.btp + pp]; t < prog[a.btp + pp + 1]; ++t)
                    bij += a.D1[(long long)prog[a.btf + t] * P + p] * bvv[t];
                const double2 v = vt[j * TPAD + lane + 1];
                ore += bij * v.y;
                oim -= bij * v.x;
            }
        }
        a.y[(long long)i * P + p] = make_double2(ore, oim);
    }
}

__global__ __launch_bounds__(256) void k_apply(ApplyArgs a) {
    extern __shared__ double2 smem[];
    // XCD-aware block → tile mapping: blocks are dispatched round-robin over the 8 XCDs;
    // the grid is a multiple of 8 and each XCD gets a contiguous band of tiles (rows).
    const int per = gridDim.x / 8;
    const int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= a.ntiles_x * a.nrows) return;
    apply_tile(a, tile, smem);
}

// Many operators in one launch: task t owns tiles [start[t], start[t+1]).
__global__ __launch_bounds__(256) void k_apply_grouped(const ApplyArgs* __restrict__ tasks,
                                                       const int* __restrict__ start, int ntask, int total) {
    extern __shared__ double2 smem[];
    const int per = gridDim.x / 8;
    const int v = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (v >= total) return;
    int lo = 0, hi = ntask - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    const ApplyArgs a = tasks[lo];
    apply_tile(a, v - start[lo], smem);
}

}  // namespace

ApplyArgs make_apply_args(const Ctx* c, const double2* x, double2* y) {
    ApplyArgs a;
    a.x = x;
    a.y = y;
    a.D2 = c->d_D2;
    a.D1 = c->d_D1;
    a.prog = c->d_prog;
    a.vals = c->d_vals;
    a.P = c->P;
    a.n = c->n;
    a.Q = c->Q;
    a.ng2 = c->K.nfield;
    a.ng1 = c->B.nfield;
    a.dim = c->dim;
    a.ih2 = 1.0 / (c->h * c->h);
    a.kpp = c->kprog_pairptr;
    a.kpj = c->kprog_pairj;
    a.ktp = c->kprog_termptr;
    a.ktf = c->kprog_termfield;
    a.bpp = c->bprog_pairptr;
    a.bpj = c->bprog_pairj;
    a.btp = c->bprog_termptr;
    a.btf = c->bprog_termfield;
    a.kv = c->kvals_off;
    a.bv = c->bvals_off;
    a.csl_beta = c->op_csl_beta;
    a.ntiles_x = (c->n + TILE - 1) / TILE;
    a.nrows = c->dim == 2 ? c->n : 1;
    a.KF = c->d_kf;
    a.k0 = c->kbar;
    a.K0 = c->d_k0;
    a.ih = 1.0 / c->h;
    return a;
}

size_t apply_lds_bytes(int Q, int ng2) { return (size_t)Q * TPAD * sizeof(double2) + (size_t)ng2 * TILE * sizeof(double); }

static int set_lds_attr() {
    // once per process (thread-safe initialisation of a function-local static)
    static const hipError_t e = [] {
        hipError_t r = hipFuncSetAttribute((const void*)k_apply, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (r == hipSuccess)
            r = hipFuncSetAttribute((const void*)k_apply_grouped, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        return r;
    }();
    SG_HIP(e);
    return SG_OK;
}

int launch_apply_grouped(const ApplyArgs* d_tasks, const int* d_start, int ntask, int total, size_t lds,
                         double bytes, hipStream_t st) {
    if (ntask <= 0 || total <= 0) return SG_OK;
    if (lds > 160 * 1024) return fail(SG_EINVAL, "sg_apply: Q too large for the LDS tile");
    int rc = set_lds_attr();
    if (rc) return rc;
    KScope ks(SG_K_APPLY, bytes, st);
    hipLaunchKernelGGL(k_apply_grouped, dim3(((total + 7) / 8) * 8), dim3(256), lds, st, d_tasks, d_start, ntask,
                       total);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

bool apply_available(const Ctx* c, double csl_beta) {
    ApplyArgs a = make_apply_args(c, nullptr, nullptr);   // null x: the dispatchers only answer
    a.csl_beta = csl_beta;
    const int sv = c->s, rv = c->degree;
    if (c->use_spec_apply && (dispatch_spec_g0(sv, rv, a, 0) || dispatch_spec_g1(sv, rv, a, 0) ||
                              dispatch_spec_g2(sv, rv, a, 0) || dispatch_spec_g3(sv, rv, a, 0) ||
                              dispatch_spec_g4(sv, rv, a, 0)))
        return true;
    return apply_lds_bytes(c->Q, c->K.nfield) <= 160 * 1024;
}

int launch_apply(const Ctx* c, const double2* x, double2* y, hipStream_t st) {
    if (!x || !y) return fail(SG_EINVAL, "sg_apply: null vector");
    if (x == y) return fail(SG_EINVAL, "sg_apply: x and y must not alias");
    const ApplyArgs a = make_apply_args(c, x, y);
    if (c->use_spec_apply) {
        KScope ks(SG_K_APPLY, (double)c->P * (32.0 * c->Q + 8.0 * c->s), st);
        const int sv = c->s, rv = c->degree;
        if (dispatch_spec_g0(sv, rv, a, st) || dispatch_spec_g1(sv, rv, a, st) ||
            dispatch_spec_g2(sv, rv, a, st) || dispatch_spec_g3(sv, rv, a, st) || dispatch_spec_g4(sv, rv, a, st)) {
            SG_HIP(hipGetLastError());
            return SG_OK;
        }
    }
    const size_t lds = apply_lds_bytes(c->Q, c->K.nfield);
    if (lds > 160 * 1024) return fail(SG_EINVAL, "sg_apply: Q too large for the LDS tile");
    int rc = set_lds_attr();
    if (rc) return rc;
    const int nblk = ((a.ntiles_x * a.nrows + 7) / 8) * 8;
    KScope ks(SG_K_APPLY, (double)c->P * (32.0 * c->Q + 8.0 * c->K.nfield), st);
    hipLaunchKernelGGL(k_apply, dim3(nblk), dim3(256), lds, st, a);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

}  // namespace sgi
