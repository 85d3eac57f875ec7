// Vector kernels of the Krylov drivers (HBM-bound, FP64 complex).
//
//  multidot   partial[b][k] = Σ_{i in block b} conj(V_k[i]) · w[i]        (first stage)
//  reduce     out[k] = scale[k] · Σ_b partial[b][k]                        (second stage)
//  axpy       w[i] -= Σ_k V_k[i] · scale[k] · coef[k]
//  norm2      partial[b] = Σ_{i in block b} |x[i]|²
//  lincomb    x[i] += Σ_k V_k[i] · scale[k] · coef[k]
//
// The basis vectors are kept unnormalised: v_k = scale[k] · V_k, so a new Arnoldi
// vector never needs a separate normalisation pass.  Reductions are two-stage with a
// fixed order (no atomics), so results are bitwise repeatable.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sg_internal.h"

namespace sgi {

namespace {

constexpr int RB = 256;      // threads per block
constexpr int KG = 16;       // basis vectors per register group
constexpr int MAXBLK = 2048; // first-stage blocks

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-reduce KG complex values; thread 0 of the block ends up with the totals in red[].
__device__ __forceinline__ void block_reduce(double2 (&acc)[KG], double2* red /* [4][KG] */) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < KG; ++k) {
        acc[k].x = wave_sum(acc[k].x);
        acc[k].y = wave_sum(acc[k].y);
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < KG; ++k) red[wv * KG + k] = acc[k];
    }
    __syncthreads();
    if (threadIdx.x < KG) {
        double2 s = red[threadIdx.x];
        for (int w = 1; w < RB / 64; ++w) {
            s.x += red[w * KG + threadIdx.x].x;
            s.y += red[w * KG + threadIdx.x].y;
        }
        red[threadIdx.x] = s;
    }
    __syncthreads();
}

__global__ __launch_bounds__(RB) void k_multidot(long long n, int nv, const double2* __restrict__ V, long long ldv,
                                                 const double2* __restrict__ w, double2* __restrict__ partial) {
    __shared__ double2 red[(RB / 64) * KG];
    const long long stride = (long long)gridDim.x * RB;
    for (int kg = 0; kg < nv; kg += KG) {
        double2 acc[KG];
#pragma unroll
        for (int k = 0; k < KG; ++k) acc[k] = make_double2(0.0, 0.0);
        for (long long i = (long long)blockIdx.x * RB + threadIdx.x; i < n; i += stride) {
            const double2 wi = w[i];
#pragma unroll
            for (int k = 0; k < KG; ++k) {
                if (kg + k < nv) {
                    const double2 v = V[(long long)(kg + k) * ldv + i];
                    acc[k].x += v.x * wi.x + v.y * wi.y;   // conj(v) * w
                    acc[k].y += v.x * wi.y - v.y * wi.x;
                }
            }
        }
        block_reduce(acc, red);
        if (threadIdx.x < KG && kg + threadIdx.x < nv)
            partial[(long long)blockIdx.x * nv + kg + threadIdx.x] = red[threadIdx.x];
        __syncthreads();
    }
}

__global__ __launch_bounds__(RB) void k_norm2(long long n, const double2* __restrict__ x, double2* __restrict__ partial) {
    __shared__ double red[RB / 64];
    double s = 0.0;
    for (long long i = (long long)blockIdx.x * RB + threadIdx.x; i < n; i += (long long)gridDim.x * RB) {
        const double2 v = x[i];
        s += v.x * v.x + v.y * v.y;
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < RB / 64; ++w) t += red[w];
        partial[blockIdx.x] = make_double2(t, 0.0);
    }
}

// One block per output coefficient k; mode 0: scaled complex sum, mode 1: sqrt of real sum
// (and, when inv is given, its reciprocal: the lazy scale of the next basis vector).
__global__ __launch_bounds__(RB) void k_reduce(int nblocks, int nv, const double2* __restrict__ partial,
                                               const double* __restrict__ scale, double2* __restrict__ out, int mode,
                                               double* __restrict__ inv) {
    __shared__ double2 red[RB / 64];
    const int k = blockIdx.x;
    double sx = 0.0, sy = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += RB) {
        const double2 p = partial[(long long)b * nv + k];
        sx += p.x;
        sy += p.y;
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_double2(sx, sy);
    __syncthreads();
    if (threadIdx.x == 0) {
        double tx = 0.0, ty = 0.0;
        for (int w = 0; w < RB / 64; ++w) {
            tx += red[w].x;
            ty += red[w].y;
        }
        if (mode == 1) {
            const double nrm = sqrt(tx);
            out[k] = make_double2(nrm, 0.0);
            if (inv) *inv = 1.0 / nrm;
        } else {
            const double s = scale ? scale[k] : 1.0;
            out[k] = make_double2(s * tx, s * ty);
        }
    }
}

// w[i] = w[i] + sign · Σ_k V_k[i] · scale[k] · coef[k]
__global__ __launch_bounds__(RB) void k_axpy(long long n, int nv, const double2* __restrict__ V, long long ldv,
                                             const double* __restrict__ scale, const double2* __restrict__ coef,
                                             double2* __restrict__ w, double sign) {
    __shared__ double2 c[512];
    for (int k = threadIdx.x; k < nv; k += RB) {
        const double s = (scale ? scale[k] : 1.0) * sign;
        c[k] = make_double2(coef[k].x * s, coef[k].y * s);
    }
    __syncthreads();
    for (long long i = (long long)blockIdx.x * RB + threadIdx.x; i < n; i += (long long)gridDim.x * RB) {
        double2 acc = w[i];
        for (int k = 0; k < nv; ++k) {
            const double2 v = V[(long long)k * ldv + i];
            const double2 ck = c[k];
            acc.x += v.x * ck.x - v.y * ck.y;
            acc.y += v.x * ck.y + v.y * ck.x;
        }
        w[i] = acc;
    }
}

__global__ __launch_bounds__(RB) void k_axpby(long long n, double2 a, const double2* __restrict__ x, double2 b,
                                              const double2* __restrict__ y, double2* __restrict__ out) {
    for (long long i = (long long)blockIdx.x * RB + threadIdx.x; i < n; i += (long long)gridDim.x * RB) {
        const double2 xv = x[i];
        double2 r = make_double2(a.x * xv.x - a.y * xv.y, a.x * xv.y + a.y * xv.x);
        if (y) {
            const double2 yv = y[i];
            r.x += b.x * yv.x - b.y * yv.y;
            r.y += b.x * yv.y + b.y * yv.x;
        }
        out[i] = r;
    }
}

// CGS2 passes with the basis split across the waves of a block: wave wv owns the vectors
// k = wv, wv+4, wv+8, ... (at most NVW of them) over a chunk of 64 consecutive elements, so
// each lane keeps only its NVW basis values and accumulators in registers.
//   MODE 0  projection:  partial[b][k] = Σ conj(V_k[i]) w[i]
//   MODE 1  update + next projection:  w ← w − Σ_k c_k V_k (c_k = scale_k coef_k), then
//           partial[b][k] = Σ conj(V_k[i]) w_new[i] with the V_k values still in registers
//   MODE 2  update + squared norm:  partial[b][0] = Σ |w_new[i]|²
// The four per-wave partial sums of the update meet in a double-buffered LDS array, so one
// barrier per chunk suffices; every wave forms the same w_new, wave 0 stores it.
template <int NVW, int MODE>
__device__ __forceinline__ void cgs_block(long long n, int nv, const double2* __restrict__ V, long long ldv,
                                          const double* __restrict__ scale, const double2* __restrict__ coef,
                                          double2* __restrict__ w, double2* __restrict__ partial, int lb, int nb) {
    __shared__ double2 part[2][RB / 64][64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double2 c[NVW];
    int nk = 0;
#pragma unroll
    for (int m = 0; m < NVW; ++m) {
        const int k = wv + 4 * m;
        if (k < nv) {
            nk = m + 1;
            if (MODE != 0) {
                const double sk = -(scale ? scale[k] : 1.0);
                c[m] = make_double2(coef[k].x * sk, coef[k].y * sk);
            }
        }
    }
    double2 acc[NVW];
#pragma unroll
    for (int m = 0; m < NVW; ++m) acc[m] = make_double2(0.0, 0.0);
    double nrm = 0.0;
    int buf = 0;
    for (long long c0 = (long long)lb * 64; c0 < n; c0 += (long long)nb * 64, buf ^= 1) {
        const long long i = c0 + lane;
        const bool ok = i < n;
        double2 v[NVW];
#pragma unroll
        for (int m = 0; m < NVW; ++m)
            v[m] = (m < nk && ok) ? V[(long long)(wv + 4 * m) * ldv + i] : make_double2(0.0, 0.0);
        if constexpr (MODE == 0) {
            const double2 wi = ok ? w[i] : make_double2(0.0, 0.0);
#pragma unroll
            for (int m = 0; m < NVW; ++m) {
                acc[m].x = fma(v[m].x, wi.x, fma(v[m].y, wi.y, acc[m].x));
                acc[m].y = fma(v[m].x, wi.y, fma(-v[m].y, wi.x, acc[m].y));
            }
        } else {
            // every wave reads w[i] before the barrier: wave 0 stores the updated value after
            // it, so a read behind the barrier could see the new value instead of the old one
            double2 wn = ok ? w[i] : make_double2(0.0, 0.0);
            double2 p = make_double2(0.0, 0.0);
#pragma unroll
            for (int m = 0; m < NVW; ++m)
                if (m < nk) {
                    p.x = fma(v[m].x, c[m].x, fma(-v[m].y, c[m].y, p.x));
                    p.y = fma(v[m].x, c[m].y, fma(v[m].y, c[m].x, p.y));
                }
            part[buf][wv][lane] = p;
            __syncthreads();
#pragma unroll
            for (int q = 0; q < RB / 64; ++q) {
                wn.x += part[buf][q][lane].x;
                wn.y += part[buf][q][lane].y;
            }
            if (wv == 0 && ok && nv > 0) w[i] = wn;
            if constexpr (MODE == 1) {
#pragma unroll
                for (int m = 0; m < NVW; ++m) {
                    acc[m].x = fma(v[m].x, wn.x, fma(v[m].y, wn.y, acc[m].x));
                    acc[m].y = fma(v[m].x, wn.y, fma(-v[m].y, wn.x, acc[m].y));
                }
            } else {
                if (wv == 0) nrm = fma(wn.x, wn.x, fma(wn.y, wn.y, nrm));
            }
        }
    }
    if constexpr (MODE == 2) {
        nrm = wave_sum(nrm);
        if (wv == 0 && lane == 0) partial[lb] = make_double2(nrm, 0.0);
    } else {
#pragma unroll
        for (int m = 0; m < NVW; ++m) {
            const double sx = wave_sum(acc[m].x), sy = wave_sum(acc[m].y);
            if (lane == 0 && m < nk) partial[(long long)lb * nv + wv + 4 * m] = make_double2(sx, sy);
        }
    }
}

template <int NVW, int MODE>
__global__ __launch_bounds__(RB) void k_cgs(long long n, int nv, const double2* __restrict__ V, long long ldv,
                                            const double* __restrict__ scale, const double2* __restrict__ coef,
                                            double2* __restrict__ w, double2* __restrict__ partial) {
    cgs_block<NVW, MODE>(n, nv, V, ldv, scale, coef, w, partial, blockIdx.x, gridDim.x);
}

// ---- grouped forms: one launch over the solves of a batch -------------------------------

__device__ __forceinline__ int task_of(const int* __restrict__ start, int ntask, int v) {
    int lo = 0, hi = ntask - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The three CGS2 passes of cgs_block, per task.
template <int NVW, int MODE>
__global__ __launch_bounds__(RB) void k_cgs_g(const VecTask* __restrict__ tasks, const int* __restrict__ start,
                                              int ntask) {
    const int t = task_of(start, ntask, blockIdx.x);
    const VecTask& g = tasks[t];
    cgs_block<NVW, MODE>(g.n, g.nv, g.V, g.ldv, g.scale, g.coef, g.w, g.partial, blockIdx.x - start[t], g.nblocks);
}

// One block per (task, output k): mode 0 out[k] = scale[k]·Σ_b partial[b][k] (nout = nv),
// mode 1 out[0] = sqrt(Σ_b Re partial[b][0]) (nout = 1).
__global__ __launch_bounds__(RB) void k_reduce_g(const VecTask* __restrict__ tasks, const int* __restrict__ start,
                                                 int ntask, int mode) {
    __shared__ double2 red[RB / 64];
    const int t = task_of(start, ntask, blockIdx.x);
    const VecTask& g = tasks[t];
    const int k = blockIdx.x - start[t];
    const int nout = mode == 1 ? 1 : g.nv;
    double sx = 0.0, sy = 0.0;
    for (int b = threadIdx.x; b < g.nblocks; b += RB) {
        const double2 p = g.partial[(long long)b * nout + k];
        sx += p.x;
        sy += p.y;
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_double2(sx, sy);
    __syncthreads();
    if (threadIdx.x == 0) {
        double tx = 0.0, ty = 0.0;
        for (int w = 0; w < RB / 64; ++w) {
            tx += red[w].x;
            ty += red[w].y;
        }
        if (mode == 1) {
            g.out[0] = make_double2(sqrt(tx), 0.0);
        } else {
            const double s = g.scale ? g.scale[k] : 1.0;
            g.out[k] = make_double2(s * tx, s * ty);
        }
    }
}

// w[i] = Σ_k V_k[i] · scale[k] · coef[k]   (written, not accumulated)
template <int NV>
__global__ __launch_bounds__(RB) void k_lincomb_g(const VecTask* __restrict__ tasks, const int* __restrict__ start,
                                                  int ntask) {
    __shared__ double2 c[NV];
    const int t = task_of(start, ntask, blockIdx.x);
    const VecTask& g = tasks[t];
    const int lb = blockIdx.x - start[t];
    const int nv = g.nv;
    for (int k = threadIdx.x; k < nv; k += RB) {
        const double sk = g.scale ? g.scale[k] : 1.0;
        c[k] = make_double2(g.coef[k].x * sk, g.coef[k].y * sk);
    }
    __syncthreads();
    const long long stride = (long long)g.nblocks * RB;
    for (long long i = (long long)lb * RB + threadIdx.x; i < g.n; i += stride) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < NV; ++k)
            if (k < nv) {
                const double2 v = g.V[(long long)k * g.ldv + i];
                const double2 ck = c[k];
                acc.x = fma(v.x, ck.x, fma(-v.y, ck.y, acc.x));
                acc.y = fma(v.x, ck.y, fma(v.y, ck.x, acc.y));
            }
        g.w[i] = acc;
    }
}

// w = a x + b y (y may be null; a null x reads as zero, so that w = b y or w = 0)
__global__ __launch_bounds__(RB) void k_axpby_g(const VecTask* __restrict__ tasks, const int* __restrict__ start,
                                                int ntask) {
    const int t = task_of(start, ntask, blockIdx.x);
    const VecTask& g = tasks[t];
    const int lb = blockIdx.x - start[t];
    const long long stride = (long long)g.nblocks * RB;
    const double2 a = g.a, b = g.b;
    for (long long i = (long long)lb * RB + threadIdx.x; i < g.n; i += stride) {
        const double2 xv = g.x ? g.x[i] : make_double2(0.0, 0.0);   // no x: w = b·y, or 0
        double2 r = make_double2(a.x * xv.x - a.y * xv.y, a.x * xv.y + a.y * xv.x);
        if (g.y) {
            const double2 yv = g.y[i];
            r.x += b.x * yv.x - b.y * yv.y;
            r.y += b.x * yv.y + b.y * yv.x;
        }
        g.w[i] = r;
    }
}

// ---- delayed CGS2 (one reduction and one update pass per Arnoldi step) ------------------
//
// Step j holds the orthonormal v_0..v_{j-1} (slots 0..j-1), the candidate u_j of slot j (w_{j-1}
// after one Gram-Schmidt pass, not yet re-orthogonalised nor normalised) and w_j = A z_j,
// z_j = P^{-1} u_j (slot j+1).  One pass over the slots forms
//     a = V^H u_j,  b = V^H w_j,  α = ||u_j||²,  β = u_j^H w_j,  ω = ||w_j||²;
// the re-orthogonalisation of u_j is then ν v_j = u_j - V a with ν² = α - ||a||², the
// projection of w_j on the final basis is (b, (β - a^H b)/ν), and one more pass writes v_j and
// the next candidate u_{j+1} = w_j - V b - h v_j (dcgs_update).  Reading the basis twice per
// step instead of three times, with one coefficient exchange with the host.

// partial[b][k]: k < nv: a_k;  nv <= k < 2nv: b_{k-nv};  2nv: α;  2nv+1: β;  2nv+2: ω
// (w == nullptr: only a and α, laid out as k < nv: a_k, nv: α).  UNR grid-stride chunks per
// iteration: all their loads are issued before the first product (each lane still adds its
// chunks in grid-stride order).
template <int NVW, int UNR>
// Chunk form for more than 64 basis vectors: the block covers vectors koff .. koff+nv-1 of
// the nvt of the step (V points at vector koff) and writes their columns of the partial row;
// α, β, ω come from the chunk at koff = 0.
__device__ __forceinline__ void dcgs_reduce_block(long long n, int nv, const double2* __restrict__ V, long long ldv,
                                                  const double2* __restrict__ u, const double2* __restrict__ w,
                                                  double2* __restrict__ partial, int lb, int nblk, int nvt = -1,
                                                  int koff = 0) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool hasw = w != nullptr;
    if (nvt < 0) nvt = nv;
    const int nout = hasw ? 2 * nvt + 3 : nvt + 1;
    int nk = 0;
#pragma unroll
    for (int m = 0; m < NVW; ++m)
        if (wv + 4 * m < nv) nk = m + 1;
    double2 ca[NVW], cb[NVW];
#pragma unroll
    for (int m = 0; m < NVW; ++m) ca[m] = cb[m] = make_double2(0.0, 0.0);
    double2 sc = make_double2(0.0, 0.0);   // wave 0: α; wave 1: β; wave 2: ω
    const long long stride = (long long)nblk * 64;
    for (long long c0 = (long long)lb * 64; c0 < n; c0 += stride * UNR) {
        double2 ui[UNR], wi[UNR], vv[UNR][NVW];
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
            const long long i = c0 + q * stride + lane;
            const bool ok = i < n;
            ui[q] = ok ? u[i] : make_double2(0.0, 0.0);
            wi[q] = (ok && hasw) ? w[i] : make_double2(0.0, 0.0);
#pragma unroll
            for (int m = 0; m < NVW; ++m)
                vv[q][m] = (m < nk && ok) ? V[(long long)(wv + 4 * m) * ldv + i] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
#pragma unroll
            for (int m = 0; m < NVW; ++m) {
                if (m < nk) {
                    const double2 v = vv[q][m];
                    ca[m].x = fma(v.x, ui[q].x, fma(v.y, ui[q].y, ca[m].x));     // conj(v) u
                    ca[m].y = fma(v.x, ui[q].y, fma(-v.y, ui[q].x, ca[m].y));
                    if (hasw) {
                        cb[m].x = fma(v.x, wi[q].x, fma(v.y, wi[q].y, cb[m].x));
                        cb[m].y = fma(v.x, wi[q].y, fma(-v.y, wi[q].x, cb[m].y));
                    }
                }
            }
            if (wv == 0) sc.x = fma(ui[q].x, ui[q].x, fma(ui[q].y, ui[q].y, sc.x));
            else if (wv == 1 && hasw) {
                sc.x = fma(ui[q].x, wi[q].x, fma(ui[q].y, wi[q].y, sc.x));              // conj(u) w
                sc.y = fma(ui[q].x, wi[q].y, fma(-ui[q].y, wi[q].x, sc.y));
            } else if (wv == 2 && hasw) sc.x = fma(wi[q].x, wi[q].x, fma(wi[q].y, wi[q].y, sc.x));
        }
    }
    double2* out = partial + (long long)lb * nout;
#pragma unroll
    for (int m = 0; m < NVW; ++m) {
        const double ax = wave_sum(ca[m].x), ay = wave_sum(ca[m].y);
        double bx = 0.0, by = 0.0;
        if (hasw) {
            bx = wave_sum(cb[m].x);
            by = wave_sum(cb[m].y);
        }
        if (lane == 0 && m < nk) {
            out[koff + wv + 4 * m] = make_double2(ax, ay);
            if (hasw) out[nvt + koff + wv + 4 * m] = make_double2(bx, by);
        }
    }
    const double sx = wave_sum(sc.x), sy = wave_sum(sc.y);
    if (lane == 0 && koff == 0) {
        if (!hasw) {
            if (wv == 0) out[nvt] = make_double2(sx, 0.0);
        } else if (wv < 3) {
            out[2 * nvt + wv] = make_double2(sx, wv == 1 ? sy : 0.0);
        }
    }
}

// blockIdx.y: chunk of 64 basis vectors
template <int NVW, int UNR>
__global__ __launch_bounds__(RB) void k_dcgs_reduce(long long n, int nv, const double2* __restrict__ V, long long ldv,
                                                    const double2* __restrict__ u, const double2* __restrict__ w,
                                                    double2* __restrict__ partial) {
    const int koff = 64 * blockIdx.y;
    dcgs_reduce_block<NVW, UNR>(n, min(64, nv - koff), V + (long long)koff * ldv, ldv, u, w, partial, blockIdx.x,
                                gridDim.x, nv, koff);
}

// One block: the coefficients of step j from the reduced sums red[] (layout of k_dcgs_reduce)
// and the previous first-pass projection h1prev[0..j) of w_{j-1}.  Writes
//   rec[0..j]       the completed Hessenberg column j-1 (h1prev + a, then ν)     (j >= 1)
//   rec[j+1..2j+1]  the first-pass projection h1 of w_j on v_0..v_j             (full step)
//   rec[2j+2]       (ν, ||u_{j+1}||² predicted as ω - ||h1||²)
// and, for the update pass, cv[k] (v_j = cu_v u_j + Σ cv_k v_k), cw[k] (u_{j+1} = w_j + cu_u u_j +
// Σ cw_k v_k), cu = (cu_v, cu_u), and h1prev <- h1.  A non-positive ν² gives ν = 0 (breakdown:
// the host stops the cycle; the update then writes non-finite values into unused slots).
// Scaling: the candidate u_{j+1} is stored multiplied by s_{j+1} = 1/||u_{j+1}|| as predicted
// (Pythagoras: ||w_j||² - ||h||²), so that the vectors the preconditioner and the operator
// see stay of unit size (without it they grow like ||A P^{-1}||^j and overflow in long
// cycles of a poorly scaled operator).  The flexible relation A z_j = Σ h_ij v_i holds for
// the z_j actually used, so the coefficients of w_j need no correction; the record carries
// a and ν of u_j unscaled (divided by s_j, kept in cu[6]; s_0 = 1, the raw residual).
// Coefficients: cu[0..2] = (1/ν, -h s_{j+1}/ν, s_{j+1}) act on the stored u_j and w_j.
// kraw > 0 (more than 64 basis vectors, updated in chunks): the chunks below kraw are
// applied first with the raw coefficients cv_k = -a_k, cw_k = -b_k and cu[3..5] = (1, 0, 1),
// the last chunk then with the final ones (the algebra of the one-pass update, split).
__device__ __forceinline__ void dcgs_finalize_block(int j, int full, const double2* __restrict__ red,
                                                    double2* __restrict__ h1prev, double2* __restrict__ rec,
                                                    double2* __restrict__ cv, double2* __restrict__ cw,
                                                    double2* __restrict__ cu, int kraw = 0) {
    __shared__ double s_nu, s_hx, s_hy, s_next;
    __shared__ double red_a[RB / 64], red_bx[RB / 64], red_by[RB / 64], red_bb[RB / 64];
    const int t = threadIdx.x;
    const double sj = j == 0 ? 1.0 : cu[6].x;   // read before thread 0 rewrites it below
    const double isj = 1.0 / sj;
    // ||a||², a^H b and ||b||² over the threads
    double aa = 0.0, abx = 0.0, aby = 0.0, bb = 0.0;
    for (int k = t; k < j; k += RB) {
        const double2 a = red[k];
        aa = fma(a.x, a.x, fma(a.y, a.y, aa));
        if (full) {
            const double2 b = red[j + k];
            abx = fma(a.x, b.x, fma(a.y, b.y, abx));   // conj(a) b
            aby = fma(a.x, b.y, fma(-a.y, b.x, aby));
            bb = fma(b.x, b.x, fma(b.y, b.y, bb));
        }
    }
    aa = wave_sum(aa);
    abx = wave_sum(abx);
    aby = wave_sum(aby);
    bb = wave_sum(bb);
    if ((t & 63) == 0) {
        red_a[t >> 6] = aa;
        red_bx[t >> 6] = abx;
        red_by[t >> 6] = aby;
        red_bb[t >> 6] = bb;
    }
    __syncthreads();
    if (t == 0) {
        double A = 0.0, X = 0.0, Y = 0.0, Bq = 0.0;
        for (int q = 0; q < RB / 64; ++q) {
            A += red_a[q];
            X += red_bx[q];
            Y += red_by[q];
            Bq += red_bb[q];
        }
        const double alpha = full ? red[2 * j].x : red[j].x;
        const double nu2 = alpha - A;
        const double nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
        s_nu = nu;
        double snext = 1.0;
        if (full) {
            const double2 beta = red[2 * j + 1];
            s_hx = (beta.x - X) / nu;
            s_hy = (beta.y - Y) / nu;
            const double omega = red[2 * j + 2].x;
            const double pred = omega - (s_hx * s_hx + s_hy * s_hy) - Bq;
            snext = pred > 1e-12 * omega ? 1.0 / sqrt(pred) : (omega > 0.0 ? 1.0 / sqrt(omega) : 1.0);
            rec[2 * j + 2] = make_double2(nu * isj, pred);
        } else {
            rec[2 * j + 2] = make_double2(nu * isj, 0.0);
        }
        s_next = snext;
    }
    __syncthreads();
    const double nu = s_nu, inu = 1.0 / nu, sn = s_next;
    const double hx = full ? s_hx : 0.0, hy = full ? s_hy : 0.0;   // h1_j = v_j^H w_j
    for (int k = t; k < j; k += RB) {
        const double2 a = red[k];
        rec[k] = make_double2(h1prev[k].x + a.x * isj, h1prev[k].y + a.y * isj);   // completed column j-1
        if (k < kraw) {
            cv[k] = make_double2(-a.x, -a.y);
            if (full) cw[k] = make_double2(-red[j + k].x, -red[j + k].y);
            continue;
        }
        cv[k] = make_double2(-a.x * inu, -a.y * inu);
        if (full) {
            const double2 b = red[j + k];
            // cw_k = -(b_k - h1_j a_k / ν) s_{j+1}
            cw[k] = make_double2(-(b.x - (hx * a.x - hy * a.y) * inu) * sn, -(b.y - (hx * a.y + hy * a.x) * inu) * sn);
        }
    }
    __syncthreads();   // every h1prev read above precedes the overwrite below
    if (full) {
        for (int k = t; k < j; k += RB) {
            const double2 b = red[j + k];
            rec[j + 1 + k] = b;
            h1prev[k] = b;
        }
    }
    if (t == 0) {
        rec[j] = make_double2(nu * isj, 0.0);
        if (full) {
            rec[2 * j + 1] = make_double2(hx, hy);
            h1prev[j] = make_double2(hx, hy);
            cu[6] = make_double2(sn, 0.0);
        }
        cu[0] = make_double2(inu, 0.0);
        cu[1] = make_double2(-hx * inu * sn, -hy * inu * sn);
        cu[2] = make_double2(sn, 0.0);
        cu[3] = make_double2(1.0, 0.0);
        cu[4] = make_double2(0.0, 0.0);
        cu[5] = make_double2(1.0, 0.0);
    }
}

__global__ __launch_bounds__(RB) void k_dcgs_finalize(int j, int full, const double2* __restrict__ red,
                                                      double2* __restrict__ h1prev, double2* __restrict__ rec,
                                                      double2* __restrict__ cv, double2* __restrict__ cw,
                                                      double2* __restrict__ cu, int kraw) {
    dcgs_finalize_block(j, full, red, h1prev, rec, cv, cw, cu, kraw);
}

// v_j (into u's slot) and u_{j+1} (into w's slot): the wave-split basis of cgs_block, the
// per-wave partial sums of both combinations meeting in LDS; u (waves 0 and 1) and w (wave 1)
// are read before the barrier, wave 0 stores v_j and wave 1 stores u_{j+1} after it.  UNR
// grid-stride chunks per iteration, their loads issued together.
template <int NVW, int UNR>
__device__ __forceinline__ void dcgs_update_block(long long n, int nv, const double2* __restrict__ V, long long ldv,
                                                  double2* __restrict__ u, double2* __restrict__ w,
                                                  const double2* __restrict__ cv, const double2* __restrict__ cw,
                                                  const double2* __restrict__ cu, int lb, int nblk) {
    __shared__ double2 part[2][RB / 64][UNR][2][64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int nk = 0;
    double2 c1[NVW], c2[NVW];
#pragma unroll
    for (int m = 0; m < NVW; ++m) {
        const int k = wv + 4 * m;
        if (k < nv) {
            nk = m + 1;
            c1[m] = cv[k];
            c2[m] = cw[k];
        }
    }
    const double2 cuv = cu[0], cuu = cu[1];
    const double cww = cu[2].x;
    const long long stride = (long long)nblk * 64;
    int buf = 0;
    for (long long c0 = (long long)lb * 64; c0 < n; c0 += stride * UNR, buf ^= 1) {
        double2 vv[UNR][NVW], ui[UNR], wi[UNR];
        bool ok[UNR];
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
            const long long i = c0 + q * stride + lane;
            ok[q] = i < n;
            ui[q] = (ok[q] && wv < 2) ? u[i] : make_double2(0.0, 0.0);
            wi[q] = (ok[q] && wv == 1) ? w[i] : make_double2(0.0, 0.0);
#pragma unroll
            for (int m = 0; m < NVW; ++m)
                vv[q][m] = (m < nk && ok[q]) ? V[(long long)(wv + 4 * m) * ldv + i] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
            double2 p1 = make_double2(0.0, 0.0), p2 = make_double2(0.0, 0.0);
#pragma unroll
            for (int m = 0; m < NVW; ++m)
                if (m < nk) {
                    const double2 v = vv[q][m];
                    p1.x = fma(v.x, c1[m].x, fma(-v.y, c1[m].y, p1.x));
                    p1.y = fma(v.x, c1[m].y, fma(v.y, c1[m].x, p1.y));
                    p2.x = fma(v.x, c2[m].x, fma(-v.y, c2[m].y, p2.x));
                    p2.y = fma(v.x, c2[m].y, fma(v.y, c2[m].x, p2.y));
                }
            part[buf][wv][q][0][lane] = p1;
            part[buf][wv][q][1][lane] = p2;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
            if (ok[q] && wv < 2) {
                const long long i = c0 + q * stride + lane;
                double2 acc = wv == 0 ? make_double2(ui[q].x * cuv.x - ui[q].y * cuv.y, ui[q].x * cuv.y + ui[q].y * cuv.x)
                                      : make_double2(cww * wi[q].x + ui[q].x * cuu.x - ui[q].y * cuu.y,
                                                     cww * wi[q].y + ui[q].x * cuu.y + ui[q].y * cuu.x);
#pragma unroll
                for (int p = 0; p < RB / 64; ++p) {
                    acc.x += part[buf][p][q][wv][lane].x;
                    acc.y += part[buf][p][q][wv][lane].y;
                }
                if (wv == 0) u[i] = acc;
                else w[i] = acc;
            }
        }
    }
}

template <int NVW, int UNR>
__global__ __launch_bounds__(RB) void k_dcgs_update(long long n, int nv, const double2* __restrict__ V, long long ldv,
                                                    double2* __restrict__ u, double2* __restrict__ w,
                                                    const double2* __restrict__ cv, const double2* __restrict__ cw,
                                                    const double2* __restrict__ cu) {
    dcgs_update_block<NVW, UNR>(n, nv, V, ldv, u, w, cv, cw, cu, blockIdx.x, gridDim.x);
}

// ---- grouped delayed CGS2 (the batched solver): one launch per phase over the instances
// of a lockstep step; the block -> task map is the prefix table of the other grouped kernels.

template <int NVW, int UNR>
__global__ __launch_bounds__(RB) void k_dcgs_reduce_g(const DcgsTask* __restrict__ tasks, const int* __restrict__ start,
                                                      int ntask) {
    const int t = task_of(start, ntask, blockIdx.x);
    const DcgsTask& g = tasks[t];
    const double2* u = g.V + (long long)g.j * g.ldv;
    dcgs_reduce_block<NVW, UNR>(g.n, g.j, g.V, g.ldv, u, g.full ? u + g.ldv : nullptr, g.partial,
                                blockIdx.x - start[t], g.nblocks);
}

// One block per (task, output k): red[k] = Σ_b partial[b][k] over the task's first-stage blocks.
__global__ __launch_bounds__(RB) void k_dcgs_sum_g(const DcgsTask* __restrict__ tasks, const int* __restrict__ start,
                                                   int ntask) {
    __shared__ double2 red[RB / 64];
    const int t = task_of(start, ntask, blockIdx.x);
    const DcgsTask& g = tasks[t];
    const int k = blockIdx.x - start[t];
    const int nout = g.full ? 2 * g.j + 3 : g.j + 1;
    double sx = 0.0, sy = 0.0;
    for (int b = threadIdx.x; b < g.nblocks; b += RB) {
        const double2 p = g.partial[(long long)b * nout + k];
        sx += p.x;
        sy += p.y;
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_double2(sx, sy);
    __syncthreads();
    if (threadIdx.x == 0) {
        double tx = 0.0, ty = 0.0;
        for (int w = 0; w < RB / 64; ++w) {
            tx += red[w].x;
            ty += red[w].y;
        }
        g.red[k] = make_double2(tx, ty);
    }
}

__global__ __launch_bounds__(RB) void k_dcgs_finalize_g(const DcgsTask* __restrict__ tasks, int ntask) {
    const DcgsTask& g = tasks[blockIdx.x];
    dcgs_finalize_block(g.j, g.full, g.red, g.h1, g.rec, g.cv, g.cw, g.cu);
}

template <int NVW, int UNR>
__global__ __launch_bounds__(RB) void k_dcgs_update_g(const DcgsTask* __restrict__ tasks, const int* __restrict__ start,
                                                      int ntask) {
    const int t = task_of(start, ntask, blockIdx.x);
    const DcgsTask& g = tasks[t];
    double2* u = const_cast<double2*>(g.V) + (long long)g.j * g.ldv;
    dcgs_update_block<NVW, UNR>(g.n, g.j, g.V, g.ldv, u, u + g.ldv, g.cv, g.cw, g.cu, blockIdx.x - start[t],
                                g.nblocks);
}

}  // namespace

int launch_dcgs_reduce(long long n, int nv, const double2* V, long long ldv, const double2* u, const double2* w,
                       double2* partial, int nblocks, double2* red, hipStream_t st) {
    if (nv > 512) return fail(SG_EINVAL, "delayed CGS2: more than 512 basis vectors");
    const int nout = w ? 2 * nv + 3 : nv + 1;
    const int nchunk = std::max(1, (nv + 63) / 64);   // chunks of 64 basis vectors (grid y)
    const int nvw = (std::min(nv, 64) + 3) / 4;
    // Grid: fewer, longer-running blocks than the other reductions. A sweep over 256 to
    // 2048 blocks on 36 MB and 351 MB vectors, one to sixteen basis vectors per wave, was
    // fastest at 1024 blocks with one vector per wave and at 512 from two on, with two
    // grid-stride chunks per iteration only at two vectors per wave (2-25 % over 2048).
    const int nb = std::min(nblocks, nvw <= 1 ? 1024 : 512);
    {
        KScope ks(SG_K_DOT, 16.0 * (nv + (w ? 2 : 1) * nchunk) * (double)n, st);
        const dim3 grid(nb, nchunk);
#define SG_DR(NVW_, UNR_)                                                                                         \
    if (nvw <= NVW_) {                                                                                            \
        hipLaunchKernelGGL((k_dcgs_reduce<NVW_, UNR_>), grid, dim3(RB), 0, st, n, nv, V, ldv, u, w, partial);     \
    } else
        SG_DR(1, 1) SG_DR(2, 2) SG_DR(4, 1) SG_DR(8, 1) SG_DR(16, 1) {
            return fail(SG_EINVAL, "delayed CGS2: more than 64 basis vectors per chunk");
        }
#undef SG_DR
        SG_HIP(hipGetLastError());
    }
    KScope ks(SG_K_NORM, 16.0 * nb * (double)nout, st);
    hipLaunchKernelGGL(k_reduce, dim3(nout), dim3(RB), 0, st, nb, nout, partial, (const double*)nullptr, red, 0,
                       (double*)nullptr);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int launch_dcgs_finalize(int j, bool full, const double2* red, double2* h1prev, double2* rec, double2* cv, double2* cw,
                         double2* cu, hipStream_t st) {
    KScope ks(SG_K_NORM, 0.0, st);
    const int kraw = j > 64 ? 64 * ((j - 1) / 64) : 0;   // the last chunk's first vector
    hipLaunchKernelGGL(k_dcgs_finalize, dim3(1), dim3(RB), 0, st, j, full ? 1 : 0, red, h1prev, rec, cv, cw, cu, kraw);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

// cu holds 7 entries (the final triple, the raw triple of the earlier chunks, the scale).
int launch_dcgs_update(long long n, int nv, const double2* V, long long ldv, double2* u, double2* w, const double2* cv,
                       const double2* cw, const double2* cu, int nblocks, hipStream_t st) {
    if (nv > 512) return fail(SG_EINVAL, "delayed CGS2: more than 512 basis vectors");
    const int nchunk = std::max(1, (nv + 63) / 64);
    KScope ks(SG_K_AXPY, 16.0 * (nv + 4 * nchunk) * (double)n, st);
    for (int c = 0; c < nchunk; ++c) {
        const int koff = 64 * c, nvc = std::min(64, nv - koff);
        const bool last = c + 1 == nchunk;
        const double2* cuc = last ? cu : cu + 3;
        const double2* Vc = V + (long long)koff * ldv;
        const int nvw = (nvc + 3) / 4;
        // 512 blocks from two vectors per wave on (the same sweep as the reduction: 3-7 %
        // over 1024-2048 blocks); with one vector per wave the full grid stays fastest
        const int nb = nvw >= 2 ? std::min(nblocks, 512) : nblocks;
#define SG_DU(NVW_, UNR_)                                                                                        \
    if (nvw <= NVW_) {                                                                                           \
        hipLaunchKernelGGL((k_dcgs_update<NVW_, UNR_>), dim3(nb), dim3(RB), 0, st, n, nvc, Vc, ldv, u, w, cv + koff, \
                           cw + koff, cuc);                                                                      \
    } else
        SG_DU(1, 1) SG_DU(2, 2) SG_DU(4, 1) SG_DU(8, 1) SG_DU(16, 1) {
            return fail(SG_EINVAL, "delayed CGS2: more than 64 basis vectors per chunk");
        }
#undef SG_DU
        SG_HIP(hipGetLastError());
    }
    return SG_OK;
}

// First-stage blocks of the reductions: about four 64-element chunks per block (short
// dependent chains for small vectors), at most MAXBLK.
int reduction_blocks(long long n) {
    long long b = (n + RB - 1) / RB;
    if (b < 1) b = 1;
    if (b > MAXBLK) b = MAXBLK;
    return (int)b;
}

static unsigned grid_for(long long n) {
    long long b = (n + RB - 1) / RB;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (unsigned)b;
}

static int launch_cgs(int mode, long long n, int nv, const double2* V, long long ldv, const double* scale,
                      const double2* coef, double2* w, double2* partial, int nblocks, hipStream_t st) {
    const int nvw = (nv + 3) / 4;
#define SG_CGS(NVW_)                                                                                          \
    if (nvw <= NVW_) {                                                                                        \
        if (mode == 0)                                                                                        \
            hipLaunchKernelGGL((k_cgs<NVW_, 0>), dim3(nblocks), dim3(RB), 0, st, n, nv, V, ldv, scale, coef, w, partial); \
        else if (mode == 1)                                                                                   \
            hipLaunchKernelGGL((k_cgs<NVW_, 1>), dim3(nblocks), dim3(RB), 0, st, n, nv, V, ldv, scale, coef, w, partial); \
        else                                                                                                  \
            hipLaunchKernelGGL((k_cgs<NVW_, 2>), dim3(nblocks), dim3(RB), 0, st, n, nv, V, ldv, scale, coef, w, partial); \
        SG_HIP(hipGetLastError());                                                                            \
        return 1;                                                                                             \
    }
    SG_CGS(1)
    SG_CGS(2)
    SG_CGS(4)
    SG_CGS(8)
    SG_CGS(16)
#undef SG_CGS
    return 0;
}

int launch_multidot(long long n, int nv, const double2* V, long long ldv, const double* scale, const double2* w,
                    double2* partial, int nblocks, hipStream_t st) {
    KScope ks(SG_K_DOT, 16.0 * (nv + 1) * (double)n, st);
    const int r = launch_cgs(0, n, nv, V, ldv, scale, nullptr, const_cast<double2*>(w), partial, nblocks, st);
    if (r < 0) return r;
    if (r == 1) return SG_OK;
    hipLaunchKernelGGL(k_multidot, dim3(nblocks), dim3(RB), 0, st, n, nv, V, ldv, w, partial);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int launch_reduce(int nblocks, int nv, const double2* partial, const double* scale, double2* out, hipStream_t st) {
    KScope ks(SG_K_NORM, 16.0 * nblocks * (double)nv, st);
    hipLaunchKernelGGL(k_reduce, dim3(nv), dim3(RB), 0, st, nblocks, nv, partial, scale, out, 0, (double*)nullptr);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int launch_reduce_norm(int nblocks, const double2* partial, double2* out, hipStream_t st, double* inv) {
    KScope ks(SG_K_NORM, 16.0 * nblocks, st);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(RB), 0, st, nblocks, 1, partial, (const double*)nullptr, out, 1, inv);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int launch_axpy_dot(long long n, int nv, const double2* V, long long ldv, const double* scale, const double2* coef,
                    double2* w, double2*, int, bool, hipStream_t st) {
    if (nv > 512) return fail(SG_EINVAL, "too many basis vectors");
    KScope ks(SG_K_AXPY, 16.0 * (nv + 2) * (double)n, st);
    hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(RB), 0, st, n, nv, V, ldv, scale, coef, w, -1.0);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int launch_lincomb(long long n, int nv, const double2* V, long long ldv, const double* scale, const double2* coef,
                   double2* x, hipStream_t st) {
    if (nv > 512) return fail(SG_EINVAL, "too many basis vectors");
    KScope ks(SG_K_AXPY, 16.0 * (nv + 2) * (double)n, st);
    hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(RB), 0, st, n, nv, V, ldv, scale, coef, x, 1.0);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

// Fused update (+ projection or + norm); returns 1 if handled, 0 if nv is above the
// largest fused size (64), negative on error.
int launch_upd(long long n, int nv, const double2* V, long long ldv, const double* scale, const double2* coef,
               double2* w, double2* partial, int nblocks, bool dot, hipStream_t st) {
    KScope ks(SG_K_AXPY, 16.0 * (nv + 2) * (double)n, st);
    return launch_cgs(dot ? 1 : 2, n, nv, V, ldv, scale, coef, w, partial, nblocks, st);
}

int launch_norm2(long long n, const double2* x, double2* partial, int nblocks, hipStream_t st) {
    KScope ks(SG_K_NORM, 16.0 * (double)n, st);
    hipLaunchKernelGGL(k_norm2, dim3(nblocks), dim3(RB), 0, st, n, x, partial);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int launch_axpby(long long n, double2 a, const double2* x, double2 b, const double2* y, double2* out, hipStream_t st) {
    KScope ks(SG_K_AXPY, (y ? 48.0 : 32.0) * (double)n, st);
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(RB), 0, st, n, a, x, b, y, out);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int launch_scale_copy(long long n, double a, const double2* x, double2* out, hipStream_t st) {
    return launch_axpby(n, make_double2(a, 0.0), x, make_double2(0.0, 0.0), nullptr, out, st);
}

}  // namespace sgi

namespace sgi {

static int launch_cgs_grouped(int mode, const VecTask* d_tasks, const int* d_start, int ntask, int total, int maxnv,
                              hipStream_t st) {
    const int nvw = (maxnv + 3) / 4;
#define SG_CGSG(NVW_)                                                                                         \
    if (nvw <= NVW_) {                                                                                        \
        if (mode == 0) hipLaunchKernelGGL((k_cgs_g<NVW_, 0>), dim3(total), dim3(RB), 0, st, d_tasks, d_start, ntask); \
        else if (mode == 1) hipLaunchKernelGGL((k_cgs_g<NVW_, 1>), dim3(total), dim3(RB), 0, st, d_tasks, d_start, ntask); \
        else hipLaunchKernelGGL((k_cgs_g<NVW_, 2>), dim3(total), dim3(RB), 0, st, d_tasks, d_start, ntask);  \
        SG_HIP(hipGetLastError());                                                                            \
        return SG_OK;                                                                                         \
    }
    SG_CGSG(1)
    SG_CGSG(2)
    SG_CGSG(4)
    SG_CGSG(8)
    SG_CGSG(16)
#undef SG_CGSG
    return fail(SG_EINVAL, "batched solve: restart length above 64");
}

int launch_multidot_grouped(const VecTask* d_tasks, const int* d_start, int ntask, int total, int maxnv, double bytes,
                            hipStream_t st) {
    if (ntask <= 0 || total <= 0) return SG_OK;
    KScope ks(SG_K_DOT, bytes, st);
    return launch_cgs_grouped(0, d_tasks, d_start, ntask, total, maxnv, st);
}

int launch_reduce_grouped(const VecTask* d_tasks, const int* d_start, int ntask, int total, int mode,
                          hipStream_t st) {
    if (ntask <= 0 || total <= 0) return SG_OK;
    KScope ks(SG_K_NORM, 0.0, st);
    hipLaunchKernelGGL(k_reduce_g, dim3(total), dim3(RB), 0, st, d_tasks, d_start, ntask, mode);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int launch_upd_grouped(const VecTask* d_tasks, const int* d_start, int ntask, int total, int maxnv, bool dot,
                       double bytes, hipStream_t st) {
    if (ntask <= 0 || total <= 0) return SG_OK;
    KScope ks(SG_K_AXPY, bytes, st);
    return launch_cgs_grouped(dot ? 1 : 2, d_tasks, d_start, ntask, total, maxnv, st);
}

int launch_lincomb_grouped(const VecTask* d_tasks, const int* d_start, int ntask, int total, int maxnv,
                           double bytes, hipStream_t st) {
    if (ntask <= 0 || total <= 0) return SG_OK;
    KScope ks(SG_K_AXPY, bytes, st);
#define SG_LCG(NV_)                                                                                   \
    if (maxnv <= NV_) {                                                                               \
        hipLaunchKernelGGL((k_lincomb_g<NV_>), dim3(total), dim3(RB), 0, st, d_tasks, d_start, ntask); \
        SG_HIP(hipGetLastError());                                                                    \
        return SG_OK;                                                                                 \
    }
    SG_LCG(8)
    SG_LCG(16)
    SG_LCG(32)
    SG_LCG(64)
#undef SG_LCG
    return fail(SG_EINVAL, "batched solve: restart length above 64");
}

int launch_dcgs_reduce_grouped(const DcgsTask* d_tasks, const int* d_start, int ntask, int total, int maxj, double bytes,
                               hipStream_t st) {
    if (ntask <= 0 || total <= 0) return SG_OK;
    KScope ks(SG_K_DOT, bytes, st);
    const int nvw = (maxj + 3) / 4;
#define SG_DRG(NVW_)                                                                                             \
    if (nvw <= NVW_) {                                                                                           \
        hipLaunchKernelGGL((k_dcgs_reduce_g<NVW_, (NVW_ == 2 ? 2 : 1)>), dim3(total), dim3(RB), 0, st, d_tasks,   \
                           d_start, ntask);                                                                      \
        SG_HIP(hipGetLastError());                                                                               \
        return SG_OK;                                                                                            \
    }
    SG_DRG(1) SG_DRG(2) SG_DRG(4) SG_DRG(8) SG_DRG(16)
#undef SG_DRG
    return fail(SG_EINVAL, "batched solve: more than 64 basis vectors");
}

int launch_dcgs_sum_grouped(const DcgsTask* d_tasks, const int* d_start, int ntask, int total, hipStream_t st) {
    if (ntask <= 0 || total <= 0) return SG_OK;
    KScope ks(SG_K_NORM, 0.0, st);
    hipLaunchKernelGGL(k_dcgs_sum_g, dim3(total), dim3(RB), 0, st, d_tasks, d_start, ntask);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int launch_dcgs_finalize_grouped(const DcgsTask* d_tasks, int ntask, hipStream_t st) {
    if (ntask <= 0) return SG_OK;
    KScope ks(SG_K_NORM, 0.0, st);
    hipLaunchKernelGGL(k_dcgs_finalize_g, dim3(ntask), dim3(RB), 0, st, d_tasks, ntask);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int launch_dcgs_update_grouped(const DcgsTask* d_tasks, const int* d_start, int ntask, int total, int maxj, double bytes,
                               hipStream_t st) {
    if (ntask <= 0 || total <= 0) return SG_OK;
    KScope ks(SG_K_AXPY, bytes, st);
    const int nvw = (maxj + 3) / 4;
#define SG_DUG(NVW_)                                                                                             \
    if (nvw <= NVW_) {                                                                                           \
        hipLaunchKernelGGL((k_dcgs_update_g<NVW_, (NVW_ == 2 ? 2 : 1)>), dim3(total), dim3(RB), 0, st, d_tasks,   \
                           d_start, ntask);                                                                      \
        SG_HIP(hipGetLastError());                                                                               \
        return SG_OK;                                                                                            \
    }
    SG_DUG(1) SG_DUG(2) SG_DUG(4) SG_DUG(8) SG_DUG(16)
#undef SG_DUG
    return fail(SG_EINVAL, "batched solve: more than 64 basis vectors");
}

int launch_axpby_grouped(const VecTask* d_tasks, const int* d_start, int ntask, int total, double bytes,
                         hipStream_t st) {
    if (ntask <= 0 || total <= 0) return SG_OK;
    KScope ks(SG_K_AXPY, bytes, st);
    hipLaunchKernelGGL(k_axpby_g, dim3(total), dim3(RB), 0, st, d_tasks, d_start, ntask);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

}  // namespace sgi
