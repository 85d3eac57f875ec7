// Mean-value (A_0) and mean-CSL (M_0) preconditioner solves (Section 5, eq. bar_A;
// eq. M with the shift on the k² term; Section 6.3 reuse of one block factorisation for
// all m+1 blocks).
//
// 2D: z = (I_Q ⊗ S(ξ̄))^{-1} r with S(ξ̄) = D⊗S_1 + S_1⊗D is solved per block by
//   (1) R' = R Ṽ             dense transform along x (complex GEMM, all Q·N rows at once),
//   (2) for every column a:  (T - i(k̄/h)E_1 + (μ_a - c) D) w_a = r'_a   along y,
//       pivoted tridiagonal LU factors precomputed in FP64 at setup,
//   (3) Z = W Ṽᵀ             inverse transform along x.
// 1D: S(ξ̄) is itself tridiagonal: step (2) alone, one system per block.
//
// The complex GEMM C = A·B with complex-interleaved rows is done as the real GEMM
// C[M×2N] = A[M×2K] · Bexp[2K×2N], Bexp[2k+c][2n+d] = [[Re, Im], [-Im, Re]](B[k][n]),
// so the interleaved complex128 buffers are used as they are.  Bexp is stored
// n-major (Bt[2n+d][2k+c]) in the compute precision.  Three arithmetic modes:
//   F64     v_mfma_f64_16x16x4f64, FP64 throughout;
//   F32     A rounded to FP32 on load, v_mfma_f32_16x16x4f32, FP32 accumulation;
//   BF16X3  A and B split into bf16 hi + lo, C += Ahi·Bhi + Ahi·Blo + Alo·Bhi with
//           v_mfma_f32_16x16x32_bf16, FP32 accumulation.
// In the two reduced-precision forms the intermediate of steps (1)-(3) is stored in FP32
// (the forward transform writes FP32, the sweep runs in FP32 with the FP64 factors rounded
// as they are loaded, the inverse transform reads FP32): the transforms round their A
// operand to FP32 in any case, and the sweep and the transforms move half the bytes.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "sg_internal.h"

namespace sgi {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

enum { MODE_F64 = 0, MODE_F32 = 1, MODE_BF16X3 = 2 };

constexpr int BK = 32;

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// LDS tiles of one K step.  BM = 32·WM rows of A, BN = 32·WN rows of Bt.
template <int MODE, int BM, int BN>
struct Lds;
template <int BM, int BN>
struct Lds<MODE_F64, BM, BN> {
    static constexpr int PAD = BK + 1;
    double a[BM * PAD];
    double b[BN * PAD];
};
template <int BM, int BN>
struct Lds<MODE_F32, BM, BN> {
    static constexpr int PAD = BK + 1;
    float a[BM * PAD];
    float b[BN * PAD];
};
template <int BM, int BN>
struct Lds<MODE_BF16X3, BM, BN> {
    static constexpr int PAD = BK + 8;
    uint16_t ahi[BM * PAD], alo[BM * PAD];
    uint16_t bhi[BN * PAD], blo[BN * PAD];
};

}  // namespace

namespace {

// One BM×BN output tile (BM = 32·WM, BN = 32·WN) by four waves in a 2×2 layout, each wave
// owning WM×WN blocks of 16×16.  Global → register prefetch of the next K step overlaps
// the MFMAs of the current one.
template <int MODE, int WM, int WN, int IO = GEMM_IO_F64>
__device__ __forceinline__ void gemm_tile(const GemmTask& g, int tile, Lds<MODE, 32 * WM, 32 * WN>& sm) {
    static_assert(MODE != MODE_F64 || IO == GEMM_IO_F64, "FP64 transforms read and write FP64");
    constexpr int BM = 32 * WM, BN = 32 * WN;
    constexpr int PAD = Lds<MODE, BM, BN>::PAD;
    const double* __restrict__ A = g.A;
    const long long lda = g.lda, ldb = g.ldb, ldc = g.ldc;
    const int M = g.M, Nc = g.Nc, Kc = g.Kc;
    const int tm = tile / g.tiles_n, tn = tile % g.tiles_n;
    const int m0 = tm * BM, n0 = tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv >> 1, wn = wv & 1;
    const int l16 = lane & 15, lq = lane >> 4;

    using acc_t = typename std::conditional<MODE == MODE_F64, d4, f4>::type;
    acc_t acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    // global → register staging: the A tile is BM×32 doubles = 16·BM double2
    constexpr int PA = BM / 16, PB64 = BN / 16, PB32 = BN / 32, PB16 = BN / 64 > 0 ? BN / 64 : 1;
    using ra_t = typename std::conditional<IO == GEMM_IO_A32, float2, double2>::type;
    ra_t ra[PA];
    double2 rb64[MODE == MODE_F64 ? PB64 : 1];
    float4 rb32[MODE == MODE_F32 ? PB32 : 1];
    uint4 rbh[PB16], rbl[PB16];

    auto load_tiles = [&](int k0) {
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            const int idx = p * 256 + tid, row = idx >> 4, k = (idx & 15) * 2;
            const int gm = m0 + row, gk = k0 + k;
            ra[p] = ra_t{0, 0};
            if (gm < M && gk < Kc) {
                if constexpr (IO == GEMM_IO_A32)   // FP32 intermediate
                    ra[p] = *reinterpret_cast<const float2*>(reinterpret_cast<const float*>(A) + (long long)gm * lda + gk);
                else
                    ra[p] = *reinterpret_cast<const double2*>(A + (long long)gm * lda + gk);
            }
        }
        if constexpr (MODE == MODE_F64) {
            const double* B = reinterpret_cast<const double*>(g.Bt0);
#pragma unroll
            for (int p = 0; p < PB64; ++p) {
                const int idx = p * 256 + tid, row = idx >> 4, k = (idx & 15) * 2;
                const int gn = n0 + row, gk = k0 + k;
                rb64[p] = (gn < Nc && gk < Kc) ? *reinterpret_cast<const double2*>(B + (long long)gn * ldb + gk)
                                               : make_double2(0.0, 0.0);
            }
        } else if constexpr (MODE == MODE_F32) {
            const float* B = reinterpret_cast<const float*>(g.Bt0);
#pragma unroll
            for (int p = 0; p < PB32; ++p) {
                const int idx = p * 256 + tid, row = idx >> 3, k = (idx & 7) * 4;
                const int gn = n0 + row, gk = k0 + k;
                // Kc is even and ldb a multiple of 4: a float4 is either fully inside or
                // straddles the end, in which case the tail lanes are read as zero.
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (gn < Nc && gk + 3 < Kc) v = *reinterpret_cast<const float4*>(B + (long long)gn * ldb + gk);
                else if (gn < Nc && gk < Kc) {
                    v.x = B[(long long)gn * ldb + gk];
                    v.y = B[(long long)gn * ldb + gk + 1];
                }
                rb32[p] = v;
            }
        } else {
            const uint16_t* Bh = reinterpret_cast<const uint16_t*>(g.Bt0);
            const uint16_t* Bl = reinterpret_cast<const uint16_t*>(g.Bt1);
#pragma unroll
            for (int p = 0; p < PB16; ++p) {
                const int idx = p * 256 + tid, row = idx >> 2, k = (idx & 3) * 8;
                const int gn = n0 + row, gk = k0 + k;
                uint4 vh = make_uint4(0, 0, 0, 0), vl = make_uint4(0, 0, 0, 0);
                if (row < BN && gn < Nc && gk < Kc) {   // ldb is padded to a multiple of 8 with zeros
                    vh = *reinterpret_cast<const uint4*>(Bh + (long long)gn * ldb + gk);
                    vl = *reinterpret_cast<const uint4*>(Bl + (long long)gn * ldb + gk);
                }
                rbh[p] = vh;
                rbl[p] = vl;
            }
        }
    };

    auto store_tiles = [&]() {
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            const int idx = p * 256 + tid, row = idx >> 4, k = (idx & 15) * 2;
            if constexpr (MODE == MODE_F64) {
                sm.a[row * PAD + k] = ra[p].x;
                sm.a[row * PAD + k + 1] = ra[p].y;
            } else if constexpr (MODE == MODE_F32) {
                sm.a[row * PAD + k] = (float)ra[p].x;
                sm.a[row * PAD + k + 1] = (float)ra[p].y;
            } else {
                const float x0 = (float)ra[p].x, x1 = (float)ra[p].y;
                const uint16_t h0 = bf16_rne(x0), h1 = bf16_rne(x1);
                sm.ahi[row * PAD + k] = h0;
                sm.ahi[row * PAD + k + 1] = h1;
                sm.alo[row * PAD + k] = bf16_rne((float)(ra[p].x - (double)bf16_to_f(h0)));
                sm.alo[row * PAD + k + 1] = bf16_rne((float)(ra[p].y - (double)bf16_to_f(h1)));
            }
        }
        if constexpr (MODE == MODE_F64) {
#pragma unroll
            for (int p = 0; p < PB64; ++p) {
                const int idx = p * 256 + tid, row = idx >> 4, k = (idx & 15) * 2;
                sm.b[row * PAD + k] = rb64[p].x;
                sm.b[row * PAD + k + 1] = rb64[p].y;
            }
        } else if constexpr (MODE == MODE_F32) {
#pragma unroll
            for (int p = 0; p < PB32; ++p) {
                const int idx = p * 256 + tid, row = idx >> 3, k = (idx & 7) * 4;
                sm.b[row * PAD + k] = rb32[p].x;
                sm.b[row * PAD + k + 1] = rb32[p].y;
                sm.b[row * PAD + k + 2] = rb32[p].z;
                sm.b[row * PAD + k + 3] = rb32[p].w;
            }
        } else {
#pragma unroll
            for (int p = 0; p < PB16; ++p) {
                const int idx = p * 256 + tid, row = idx >> 2, k = (idx & 3) * 8;
                if (row < BN) {
                    *reinterpret_cast<uint4*>(&sm.bhi[row * PAD + k]) = rbh[p];
                    *reinterpret_cast<uint4*>(&sm.blo[row * PAD + k]) = rbl[p];
                }
            }
        }
    };

    const int nk = (Kc + BK - 1) / BK;
    load_tiles(0);
    for (int kt = 0; kt < nk; ++kt) {
        __syncthreads();
        store_tiles();
        __syncthreads();
        if (kt + 1 < nk) load_tiles((kt + 1) * BK);
        if constexpr (MODE == MODE_BF16X3) {
            bf8 ah[WM], al[WM], bh[WN], bl[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                const int r = wm * (16 * WM) + i * 16 + l16;
                ah[i] = *reinterpret_cast<const bf8*>(&sm.ahi[r * PAD + lq * 8]);
                al[i] = *reinterpret_cast<const bf8*>(&sm.alo[r * PAD + lq * 8]);
            }
#pragma unroll
            for (int j = 0; j < WN; ++j) {
                const int cN = wn * (16 * WN) + j * 16 + l16;
                bh[j] = *reinterpret_cast<const bf8*>(&sm.bhi[cN * PAD + lq * 8]);
                bl[j] = *reinterpret_cast<const bf8*>(&sm.blo[cN * PAD + lq * 8]);
            }
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                }
        } else {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                using e_t = typename std::conditional<MODE == MODE_F64, double, float>::type;
                e_t av[WM], bv[WN];
#pragma unroll
                for (int i = 0; i < WM; ++i) av[i] = sm.a[(wm * (16 * WM) + i * 16 + l16) * PAD + kk + lq];
#pragma unroll
                for (int j = 0; j < WN; ++j) bv[j] = sm.b[(wn * (16 * WN) + j * 16 + l16) * PAD + kk + lq];
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < WN; ++j) {
                        if constexpr (MODE == MODE_F64)
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
                        else
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
                    }
            }
        }
    }
    // epilogue: the f32-output MFMAs leave D[4*lq + v][l16] of each 16×16 block in lane
    // (lq, l16); the f64 one leaves D[lq + 4*v][l16].
    double* __restrict__ C = g.C;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            const int col = n0 + wn * (16 * WN) + j * 16 + l16;
            if (col >= Nc) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rl = (MODE == MODE_F64) ? (lq + 4 * v) : (lq * 4 + v);
                const int row = m0 + wm * (16 * WM) + i * 16 + rl;
                if (row < M) {
                    if constexpr (IO == GEMM_IO_C32)
                        reinterpret_cast<float*>(C)[(long long)row * ldc + col] = (float)acc[i][j][v];
                    else
                        C[(long long)row * ldc + col] = (double)acc[i][j][v];
                }
            }
        }
}

// 3M complex product, FP64 or FP32: C = A·B with complex A [M][K] (interleaved FP64), B
// [K][N] given as two real n-major planes Br, Bi in the compute precision.  Per 16×16
// complex output block and K step: P1 += Ar·Br, P2 += Ai·Bi, P3 += (Ar+Ai)·(Br+Bi) on
// v_mfma_f64_16x16x4f64 (v_mfma_f32_16x16x4f32); then Re = P1 − P2, Im = P3 − P1 − P2, formed
// in FP64.  Three real products per complex multiply-add instead of the four of the
// expanded real form.  BM = 32·WM complex rows, BN = 32·WN complex columns, BK3 complex k
// per LDS stage; LDS holds the real and imaginary planes only, the sums are formed in
// registers after the LDS reads (a third less LDS traffic than staging them).
constexpr int BK3 = 16;

template <int MODE, int BM, int BN>
struct Lds3 {
    using e_t = typename std::conditional<MODE == MODE_F64, double, float>::type;
    static constexpr int PAD = BK3 + 1;
    e_t ar[BM * PAD], ai[BM * PAD];
    e_t br[BN * PAD], bi[BN * PAD];
};

template <int MODE, int WM, int WN, int IO = GEMM_IO_F64>
__device__ __forceinline__ void gemm3m_tile(const GemmTask& g, int tile, Lds3<MODE, 32 * WM, 32 * WN>& sm) {
    static_assert(MODE != MODE_F64 || IO == GEMM_IO_F64, "FP64 transforms read and write FP64");
    constexpr int BM = 32 * WM, BN = 32 * WN;
    constexpr int PAD = Lds3<MODE, BM, BN>::PAD;
    using e_t = typename Lds3<MODE, BM, BN>::e_t;
    using e2_t = typename std::conditional<MODE == MODE_F64, double2, float2>::type;
    using acc_t = typename std::conditional<MODE == MODE_F64, d4, f4>::type;
    const int M = g.M, N = g.Nc / 2, K = g.Kc / 2;   // complex sizes
    const int tm = tile / g.tiles_n, tn = tile % g.tiles_n;
    const int m0 = tm * BM, n0 = tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv >> 1, wn = wv & 1;
    const int l16 = lane & 15, lq = lane >> 4;
    const double* __restrict__ A = g.A;
    const e_t* __restrict__ Br = reinterpret_cast<const e_t*>(g.Bt0);
    const e_t* __restrict__ Bi = reinterpret_cast<const e_t*>(g.Bt1);
    const long long lda = g.lda, ldb = g.ldb;

    acc_t p1[WM][WN], p2[WM][WN], p3[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) p1[i][j] = p2[i][j] = p3[i][j] = acc_t{0, 0, 0, 0};

    // staging: A tile BM × BK3 complex (BM·BK3/256 double2 per thread); B planes BN × BK3
    // doubles each, loaded as double2 pairs along k (BN·BK3/512 pairs per thread)
    constexpr int PA = BM * BK3 / 256, PB = BN * BK3 / 512, HK = BK3 / 2;
    using ra_t = typename std::conditional<IO == GEMM_IO_A32, float2, double2>::type;
    ra_t ra[PA];
    e2_t rbr[PB], rbi[PB];
    auto load_tiles = [&](int k0) {
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            const int idx = p * 256 + tid, row = idx / BK3, k = idx % BK3;
            const int gm = m0 + row, gk = k0 + k;
            ra[p] = ra_t{0, 0};
            if (gm < M && gk < K) {
                if constexpr (IO == GEMM_IO_A32)   // FP32 intermediate
                    ra[p] = *reinterpret_cast<const float2*>(reinterpret_cast<const float*>(A) + (long long)gm * lda +
                                                             2 * gk);
                else
                    ra[p] = *reinterpret_cast<const double2*>(A + (long long)gm * lda + 2 * gk);
            }
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            const int idx = p * 256 + tid, row = idx / HK, k = (idx % HK) * 2;
            const int gn = n0 + row, gk = k0 + k;
            // K is padded to an even ld with zero columns: a pair is inside or fully zero
            const bool ok = gn < N && gk < K;
            const long long off = (long long)gn * ldb + gk;
            rbr[p] = ok ? *reinterpret_cast<const e2_t*>(Br + off) : e2_t{0, 0};
            rbi[p] = ok ? *reinterpret_cast<const e2_t*>(Bi + off) : e2_t{0, 0};
        }
    };
    auto store_tiles = [&]() {
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            const int idx = p * 256 + tid, row = idx / BK3, k = idx % BK3;
            sm.ar[row * PAD + k] = (e_t)ra[p].x;
            sm.ai[row * PAD + k] = (e_t)ra[p].y;
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            const int idx = p * 256 + tid, row = idx / HK, k = (idx % HK) * 2;
            sm.br[row * PAD + k] = rbr[p].x;
            sm.br[row * PAD + k + 1] = rbr[p].y;
            sm.bi[row * PAD + k] = rbi[p].x;
            sm.bi[row * PAD + k + 1] = rbi[p].y;
        }
    };

    const int nk = (K + BK3 - 1) / BK3;
    load_tiles(0);
    for (int kt = 0; kt < nk; ++kt) {
        __syncthreads();
        store_tiles();
        __syncthreads();
        if (kt + 1 < nk) load_tiles((kt + 1) * BK3);
#pragma unroll
        for (int kk = 0; kk < BK3; kk += 4) {
            e_t xr[WM], xi[WM], xs[WM], yr[WN], yi[WN], ys[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                const int r = (wm * (16 * WM) + i * 16 + l16) * PAD + kk + lq;
                xr[i] = sm.ar[r];
                xi[i] = sm.ai[r];
                xs[i] = xr[i] + xi[i];
            }
#pragma unroll
            for (int j = 0; j < WN; ++j) {
                const int c = (wn * (16 * WN) + j * 16 + l16) * PAD + kk + lq;
                yr[j] = sm.br[c];
                yi[j] = sm.bi[c];
                ys[j] = yr[j] + yi[j];
            }
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j) {
                    if constexpr (MODE == MODE_F64) {
                        p1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[i], yr[j], p1[i][j], 0, 0, 0);
                        p2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi[i], yi[j], p2[i][j], 0, 0, 0);
                        p3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[i], ys[j], p3[i][j], 0, 0, 0);
                    } else {
                        p1[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr[i], yr[j], p1[i][j], 0, 0, 0);
                        p2[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi[i], yi[j], p2[i][j], 0, 0, 0);
                        p3[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xs[i], ys[j], p3[i][j], 0, 0, 0);
                    }
                }
        }
    }
    // the f64 MFMA leaves D[lq + 4v][l16] of each 16×16 block in lane (lq, l16), the f32 one
    // D[4lq + v][l16]
    double* __restrict__ C = g.C;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            const int col = n0 + wn * (16 * WN) + j * 16 + l16;
            if (col >= N) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rl = (MODE == MODE_F64) ? (lq + 4 * v) : (4 * lq + v);
                const int row = m0 + wm * (16 * WM) + i * 16 + rl;
                if (row < M) {
                    const double q1 = (double)p1[i][j][v], q2 = (double)p2[i][j][v], q3 = (double)p3[i][j][v];
                    const double re = q1 - q2;
                    const double im = q3 - q1 - q2;
                    if constexpr (IO == GEMM_IO_C32)
                        *reinterpret_cast<float2*>(reinterpret_cast<float*>(C) + (long long)row * g.ldc + 2 * col) =
                            make_float2((float)re, (float)im);
                    else
                        *reinterpret_cast<double2*>(C + (long long)row * g.ldc + 2 * col) = make_double2(re, im);
                }
            }
        }
}

template <int MODE, int WM, int WN, int IO>
__global__ __launch_bounds__(256) void k_gemm3m(GemmTask g) {
    __shared__ Lds3<MODE, 32 * WM, 32 * WN> sm;
    const int per = gridDim.x / 8;
    const int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= g.tiles_m * g.tiles_n) return;
    gemm3m_tile<MODE, WM, WN, IO>(g, tile, sm);
}

// Single problem; blocks are dispatched round-robin over the 8 XCDs, so the tile index is
// remapped to give each XCD a contiguous band of tiles (shared A rows and B in its L2).
template <int MODE, int WM, int WN, int IO>
__global__ __launch_bounds__(256) void k_gemm(GemmTask g) {
    __shared__ Lds<MODE, 32 * WM, 32 * WN> sm;
    const int per = gridDim.x / 8;
    const int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= g.tiles_m * g.tiles_n) return;
    gemm_tile<MODE, WM, WN, IO>(g, tile, sm);
}

// Index of the task owning virtual block v: the largest t with start[t] <= v.
__device__ __forceinline__ int find_task(const int* __restrict__ start, int ntask, int v) {
    int lo = 0, hi = ntask - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Many problems in one launch: task t owns tiles [start[t], start[t+1]) of the
// concatenated tile list; the XCD remap keeps each problem's tiles on few XCDs.
// (IO: the element types of A and C, the same for every task of one launch.)
template <int MODE, int WM, int WN, int IO>
__global__ __launch_bounds__(256) void k_gemm_grouped(const GemmTask* __restrict__ tasks,
                                                      const int* __restrict__ start, int ntask, int total) {
    __shared__ Lds<MODE, 32 * WM, 32 * WN> sm;
    const int per = gridDim.x / 8;
    const int v = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (v >= total) return;
    const int t = find_task(start, ntask, v);
    const GemmTask g = tasks[t];
    gemm_tile<MODE, WM, WN, IO>(g, v - start[t], sm);
}

template <int MODE, int WM, int WN, int IO>
__global__ __launch_bounds__(256) void k_gemm3m_grouped(const GemmTask* __restrict__ tasks,
                                                        const int* __restrict__ start, int ntask, int total) {
    __shared__ Lds3<MODE, 32 * WM, 32 * WN> sm;
    const int per = gridDim.x / 8;
    const int v = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (v >= total) return;
    const int t = find_task(start, ntask, v);
    const GemmTask g = tasks[t];
    gemm3m_tile<MODE, WM, WN, IO>(g, v - start[t], sm);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

constexpr int CH = 8;

// Pivoted tridiagonal solve, in place, one thread per system (q, a).
//   element i of system (q,a):  X[q*sq + a*sa + i*se]
//   factor row i of system a:   f.xxx[i*f.nsys + a*fa]
__global__ __launch_bounds__(64) void k_tri(double2* __restrict__ X, TriFactors f, int len, int na, int nq,
                                            long long se, long long sa, long long sq, int fa) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)na * nq) return;
    const int a = (int)(t % na), q = (int)(t / na);
    double2* x = X + (long long)q * sq + (long long)a * sa;
    const int fs = f.nsys;
    const int fo = a * fa;
    // forward: L y = P b
    double2 cur = x[0];
    for (int i0 = 0; i0 < len - 1; i0 += CH) {
        const int cnt = min(CH, len - 1 - i0);
        double2 nb[CH], l[CH];
        uint8_t pv[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u)
            if (u < cnt) {
                nb[u] = x[(long long)(i0 + u + 1) * se];
                l[u] = f.dl[(long long)(i0 + u) * fs + fo];
                pv[u] = f.piv[(long long)(i0 + u) * fs + fo];
            }
#pragma unroll
        for (int u = 0; u < CH; ++u)
            if (u < cnt) {
                double2 out, nxt;
                if (pv[u]) {
                    out = nb[u];
                    nxt = csub(cur, cmul(l[u], nb[u]));
                } else {
                    out = cur;
                    nxt = csub(nb[u], cmul(l[u], cur));
                }
                x[(long long)(i0 + u) * se] = out;
                cur = nxt;
            }
    }
    // backward: U x = y
    double2 x1 = cmul(cur, f.dinv[(long long)(len - 1) * fs + fo]);
    x[(long long)(len - 1) * se] = x1;
    if (len < 2) return;
    double2 x0 = cmul(csub(x[(long long)(len - 2) * se], cmul(f.du1[(long long)(len - 2) * fs + fo], x1)),
                      f.dinv[(long long)(len - 2) * fs + fo]);
    x[(long long)(len - 2) * se] = x0;
    // x0 = x[i+1], x1 = x[i+2]
    for (int i0 = len - 3; i0 >= 0; i0 -= CH) {
        const int cnt = min(CH, i0 + 1);
        double2 bb[CH], u1[CH], u2[CH], di[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u)
            if (u < cnt) {
                const long long i = i0 - u;
                bb[u] = x[i * se];
                u1[u] = f.du1[i * fs + fo];
                u2[u] = f.du2[i * fs + fo];
                di[u] = f.dinv[i * fs + fo];
            }
#pragma unroll
        for (int u = 0; u < CH; ++u)
            if (u < cnt) {
                const double2 r = csub(csub(bb[u], cmul(u1[u], x0)), cmul(u2[u], x1));
                const double2 xv = cmul(r, di[u]);
                x[(long long)(i0 - u) * se] = xv;
                x1 = x0;
                x0 = xv;
            }
    }
}

// Segmented pivoted tridiagonal solve (same arithmetic as k_tri, in parallel over row
// segments).  Thread (k, system) owns rows [k·L, k·L+L) (L <= SEGL) of one system and
// keeps them in registers.  Forward: run the segment with a zero entering value (segment 0
// starts from b_0); a log2(K)-round scan in LDS over the segments' affine maps (forward
// propagator, local end value) gives every segment its exact entering value; rerun and
// keep y_i/u_ii.  Backward: the same with the 2-vector state (x_{i}, x_{i+1}) and the 2x2
// propagators, as a suffix scan.  Data is read once and written once.
// Componentwise select (a ternary on the vector struct can end up as a select of
// addresses of stack copies).
__device__ __forceinline__ double2 csel(bool c, double2 a, double2 b) {
    return make_double2(c ? a.x : b.x, c ? a.y : b.y);
}
// The same row index, made to depend on v: the address formed from it, and the load, come
// only after v is known, so the factor prefetches stay at the distance written (instead of
// their addresses or loads being hoisted together and kept live through a pass) and each
// pass reloads its rows.
__device__ __forceinline__ int after(int i, double v) {
    asm volatile("" : "+v"(i) : "v"(v));
    return i;
}
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {   // a*b + c
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
// The same in FP32, for the sweep over the FP32 intermediate of the reduced-precision forms
// (the factors stay FP64 in memory and are rounded as they are loaded).
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 csel(bool c, float2 a, float2 b) {
    return make_float2(c ? a.x : b.x, c ? a.y : b.y);
}
__device__ __forceinline__ int after(int i, float v) {
    asm volatile("" : "+v"(i) : "v"(v));
    return i;
}
__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c) {
    return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}
template <typename T2>
__device__ __forceinline__ T2 fac(const double2& v);
template <>
__device__ __forceinline__ double2 fac<double2>(const double2& v) { return v; }
template <>
__device__ __forceinline__ float2 fac<float2>(const double2& v) { return make_float2((float)v.x, (float)v.y); }

// LDS of the segment joins, one scan round at a time.  The propagators depend on the system
// only, the carried values also on the right-hand side: the forward scan uses planes 0
// (propagator) and 1..NR (values), the backward one planes 0..3 (2×2 propagator) and
// 4..4+2NR-1 (2-vector values).
template <int NR, typename T2>
struct TriLds {
    T2 p[4 + 2 * NR][256];
};

// Block → (systems, right-hand sides).  With at least SYS systems per right-hand side a
// block takes SYS consecutive systems a and NR consecutive right-hand sides q (each
// thread solves its segment for all NR, sharing the factor loads), and consecutive blocks
// step through q first: the blocks that share a set of factor rows run together and find
// them in L2.  Otherwise (one system, 1D; NR = 1) a block takes SYS consecutive (a, q).
__host__ __device__ inline long long tri_blocks(int na, int nq, int K, int NR) {
    const int SYS = 256 / K;
    if (na >= SYS) return (long long)((na + SYS - 1) / SYS) * ((nq + NR - 1) / NR);
    return ((long long)na * nq + SYS - 1) / SYS;
}

template <int SEGL, int NR, typename T2>
__device__ __forceinline__ void tri_seg_block(T2* __restrict__ X, const TriFactors& f, int len, int na,
                                              int nq, long long se, long long sa, long long sq, int fa, int blk,
                                              TriLds<NR, T2>& sm) {
    const int K = f.K, L = f.L, SYS = 256 / K;
    const int tid = threadIdx.x, k = tid / SYS, sl = tid - k * SYS;
    int a, q0;
    bool valid;
    if (na >= SYS) {
        const int nqb = (nq + NR - 1) / NR;
        q0 = (blk % nqb) * NR;
        a = (blk / nqb) * SYS + sl;
        valid = a < na;
    } else {   // NR == 1
        const long long sysg = (long long)blk * SYS + sl;
        valid = sysg < (long long)na * nq;
        a = (int)(sysg % na);
        q0 = (int)(sysg / na);
    }
    if (!valid) a = q0 = 0;   // in-range reads; nothing is stored
    bool qok[NR];
    T2* x[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        qok[r] = valid && q0 + r < nq;
        x[r] = X + (long long)(qok[r] ? q0 + r : q0) * sq + (long long)a * sa;
    }
    const int fs = f.nsys;
    // factor row i of this system: ptr[i * fs]
    const double2* __restrict__ dl = f.dl + a * fa;
    const double2* __restrict__ dinv = f.dinv + a * fa;
    const double2* __restrict__ u1p = f.u1p + a * fa;
    const double2* __restrict__ u2p = f.u2p + a * fa;
    const int s0 = k * L, e0 = min(s0 + L, len);
    const T2 zero = T2{0, 0};
    const T2 ph = fac<T2>(f.phi[(long long)k * fs + a * fa]);
    const uint32_t pm = f.pivm[(long long)k * fs + a * fa];
    T2 b[NR][SEGL + 1];
#pragma unroll
    for (int u = 0; u <= SEGL; ++u) {
        const int i = s0 + u;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            b[r][u] = zero;
            if (qok[r] && u <= L && i < len) b[r][u] = x[r][(long long)i * se];
        }
    }
    // The row loops below read the factor rows PF rows ahead of their use, outside the
    // per-row conditions and from clamped, always valid rows, so that a row step never
    // waits for its own factor load.
    constexpr int PF = NR == 2 ? 2 : 4;   // two right-hand sides: fewer registers, three waves per SIMD
    const int ldl = max(len - 2, 0), lrow = len - 1;
    auto rdl = [&](int i) { return (long long)min(i, ldl) * fs; };    // row i of dl, clamped
    auto rrow = [&](int i) { return (long long)min(i, lrow) * fs; };  // row i of the others
    // forward, local run (segment 0 starts from b_0, the others from zero)
    T2 cur[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) cur[r] = csel(k == 0, b[r][0], zero);
    T2 pl[PF], pd[PF];
#pragma unroll
    for (int d = 0; d < PF; ++d) pl[d] = fac<T2>(dl[rdl(s0 + d)]);
#pragma unroll
    for (int u = 0; u < SEGL; ++u) {
        const int i = s0 + u;
        const T2 l = pl[u % PF];
        if (u + PF < SEGL) pl[u % PF] = fac<T2>(dl[rdl(after(s0 + u + PF, cur[0].x))]);
        if (i < e0 && i <= len - 2) {
            const bool pv = (pm >> u) & 1u;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const T2 nb = b[r][u + 1];
                cur[r] = csub(csel(pv, cur[r], nb), cmul(l, csel(pv, nb, cur[r])));
            }
        }
    }
    // inclusive scan over the segments of the affine maps c -> φ_k c + t_k (segment 0's
    // map is constant): afterwards T is the exact value leaving segment k
    T2 P = csel(k == 0, zero, ph), T[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) T[r] = cur[r];
    for (int d = 1; d < K; d <<= 1) {
        sm.p[0][tid] = P;
#pragma unroll
        for (int r = 0; r < NR; ++r) sm.p[1 + r][tid] = T[r];
        __syncthreads();
        if (k >= d) {
            const T2 Pp = sm.p[0][tid - d * SYS];
#pragma unroll
            for (int r = 0; r < NR; ++r) T[r] = cfma(P, sm.p[1 + r][tid - d * SYS], T[r]);
            P = cmul(P, Pp);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) sm.p[1 + r][tid] = T[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) cur[r] = csel(k == 0, b[r][0], sm.p[1 + r][max(tid - SYS, 0)]);
#pragma unroll
    for (int d = 0; d < PF; ++d) {
        pl[d] = fac<T2>(dl[rdl(after(s0 + d, cur[0].x))]);
        pd[d] = fac<T2>(dinv[rrow(after(s0 + d, cur[0].x))]);
    }
#pragma unroll
    for (int u = 0; u < SEGL; ++u) {
        const int i = s0 + u;
        const T2 l = pl[u % PF], di = pd[u % PF];
        if (u + PF < SEGL) {
            pl[u % PF] = fac<T2>(dl[rdl(after(s0 + u + PF, cur[0].x))]);
            pd[u % PF] = fac<T2>(dinv[rrow(after(s0 + u + PF, cur[0].x))]);
        }
        if (i < e0) {
            if (i <= len - 2) {
                const bool pv = (pm >> u) & 1u;
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const T2 nb = b[r][u + 1];
                    b[r][u] = cmul(csel(pv, nb, cur[r]), di);
                    cur[r] = csub(csel(pv, cur[r], nb), cmul(l, csel(pv, nb, cur[r])));
                }
            } else {
#pragma unroll
                for (int r = 0; r < NR; ++r) b[r][u] = cmul(cur[r], di);
            }
        }
    }
    // backward, local run with a zero entering state
    const double2* ps = f.psi + ((long long)k * fs + a * fa) * 4;
    T2 M00 = fac<T2>(ps[0]), M01 = fac<T2>(ps[1]), M10 = fac<T2>(ps[2]), M11 = fac<T2>(ps[3]);
    T2 x1[NR], x2[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) x1[r] = x2[r] = zero;
#pragma unroll
    for (int d = 0; d < PF; ++d) {
        pl[d] = fac<T2>(u1p[rrow(after(s0 + SEGL - 1 - d, b[0][0].x))]);
        pd[d] = fac<T2>(u2p[rrow(after(s0 + SEGL - 1 - d, b[0][0].x))]);
    }
#pragma unroll
    for (int u = SEGL - 1; u >= 0; --u) {
        const int i = s0 + u, slot = (SEGL - 1 - u) % PF;
        const T2 w1 = pl[slot], w2 = pd[slot];
        if (u - PF >= 0) {
            pl[slot] = fac<T2>(u1p[rrow(after(s0 + u - PF, x1[0].x))]);
            pd[slot] = fac<T2>(u2p[rrow(after(s0 + u - PF, x1[0].x))]);
        }
        if (i < e0) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const T2 xi = csub(csub(b[r][u], cmul(w1, x1[r])), cmul(w2, x2[r]));
                x2[r] = x1[r];
                x1[r] = xi;
            }
        }
    }
    // suffix scan of the affine maps G -> Ψ_k G + g_k (the last segment's map is
    // constant): afterwards (V0, V1) is the exact state at the start of segment k
    if (k == K - 1) M00 = M01 = M10 = M11 = zero;
    T2 V0[NR], V1[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        V0[r] = x1[r];
        V1[r] = x2[r];
    }
    __syncthreads();   // every thread has read the forward entering values
    for (int d = 1; d < K; d <<= 1) {
        sm.p[0][tid] = M00;
        sm.p[1][tid] = M01;
        sm.p[2][tid] = M10;
        sm.p[3][tid] = M11;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            sm.p[4 + 2 * r][tid] = V0[r];
            sm.p[5 + 2 * r][tid] = V1[r];
        }
        __syncthreads();
        if (k + d < K) {
            const int o = tid + d * SYS;
            const T2 N00 = sm.p[0][o], N01 = sm.p[1][o], N10 = sm.p[2][o], N11 = sm.p[3][o];
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const T2 W0 = sm.p[4 + 2 * r][o], W1 = sm.p[5 + 2 * r][o];
                V0[r] = cfma(M00, W0, cfma(M01, W1, V0[r]));
                V1[r] = cfma(M10, W0, cfma(M11, W1, V1[r]));
            }
            const T2 R00 = cfma(M00, N00, cmul(M01, N10)), R01 = cfma(M00, N01, cmul(M01, N11));
            const T2 R10 = cfma(M10, N00, cmul(M11, N10)), R11 = cfma(M10, N01, cmul(M11, N11));
            M00 = R00; M01 = R01; M10 = R10; M11 = R11;
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        sm.p[4 + 2 * r][tid] = V0[r];
        sm.p[5 + 2 * r][tid] = V1[r];
    }
    __syncthreads();
    const int nxt_seg = min(tid + SYS, 255);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        x1[r] = csel(k == K - 1, zero, sm.p[4 + 2 * r][nxt_seg]);
        x2[r] = csel(k == K - 1, zero, sm.p[5 + 2 * r][nxt_seg]);
    }
#pragma unroll
    for (int d = 0; d < PF; ++d) {
        pl[d] = fac<T2>(u1p[rrow(after(s0 + SEGL - 1 - d, x1[0].x))]);
        pd[d] = fac<T2>(u2p[rrow(after(s0 + SEGL - 1 - d, x1[0].x))]);
    }
#pragma unroll
    for (int u = SEGL - 1; u >= 0; --u) {
        const int i = s0 + u, slot = (SEGL - 1 - u) % PF;
        const T2 w1 = pl[slot], w2 = pd[slot];
        if (u - PF >= 0) {
            pl[slot] = fac<T2>(u1p[rrow(after(s0 + u - PF, x1[0].x))]);
            pd[slot] = fac<T2>(u2p[rrow(after(s0 + u - PF, x1[0].x))]);
        }
        if (i < e0) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const T2 xi = csub(csub(b[r][u], cmul(w1, x1[r])), cmul(w2, x2[r]));
                if (qok[r]) x[r][(long long)i * se] = xi;
                x2[r] = x1[r];
                x1[r] = xi;
            }
        }
    }
}

// One block of 256 threads per SYS systems (× NR right-hand sides); the XCD remap keeps
// consecutive virtual blocks (the right-hand sides of one set of systems) on one XCD.
template <int SEGL, int NR, typename T2>
__global__ __launch_bounds__(256) void k_tri_seg(T2* __restrict__ X, TriFactors f, int len, int na, int nq,
                                                 long long se, long long sa, long long sq, int fa, int total) {
    __shared__ TriLds<NR, T2> sm;
    const int per = gridDim.x / 8;
    const int v = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (v >= total) return;
    tri_seg_block<SEGL, NR, T2>(X, f, len, na, nq, se, sa, sq, fa, v, sm);
}

// (T2: float2 when every task's X is an FP32 intermediate.)
template <int SEGL, int NR, typename T2>
__global__ __launch_bounds__(256) void k_tri_seg_grouped(const TriTask* __restrict__ tasks,
                                                         const int* __restrict__ start, int ntask, int total) {
    __shared__ TriLds<NR, T2> sm;
    const int per = gridDim.x / 8;
    const int v = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (v >= total) return;
    const int t = find_task(start, ntask, v);
    const TriTask& g = tasks[t];
    tri_seg_block<SEGL, NR, T2>(reinterpret_cast<T2*>(g.X), g.f, g.len, g.na, g.nq, g.se, g.sa, g.sq, g.fa,
                                v - start[t], sm);
}

static inline uint16_t host_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
static inline float host_bf16_f(uint16_t b) {
    uint32_t u = ((uint32_t)b) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

}  // namespace

int bexp_ld(int n) { return ((2 * n + 7) / 8) * 8; }

// Bt[2n+d][2k+c] = Bexp[2k+c][2n+d] for the complex matrix B[k][n] (k, n < N).
static void expand_bt(int N, const std::vector<cplx>& B /* [k][n] */, std::vector<double>& out, int ld) {
    out.assign((size_t)2 * N * ld, 0.0);
    for (int k = 0; k < N; ++k)
        for (int n = 0; n < N; ++n) {
            const cplx b = B[(size_t)k * N + n];
            out[(size_t)(2 * n) * ld + 2 * k] = b.real();
            out[(size_t)(2 * n) * ld + 2 * k + 1] = -b.imag();
            out[(size_t)(2 * n + 1) * ld + 2 * k] = b.imag();
            out[(size_t)(2 * n + 1) * ld + 2 * k + 1] = b.real();
        }
}

// 3M planes of the complex N×N matrix B[k][n]: n-major [n][k] rows of ld values (zero
// padded), Re and Im one after the other, in FP64 and in FP32.
static int upload_planes(DenseB& d, int N, const std::vector<cplx>& B, int ld) {
    const size_t plane = (size_t)N * ld;
    std::vector<double> h(2 * plane, 0.0);
    for (int k = 0; k < N; ++k)
        for (int n = 0; n < N; ++n) {
            const cplx b = B[(size_t)k * N + n];
            h[(size_t)n * ld + k] = b.real();
            h[plane + (size_t)n * ld + k] = b.imag();
        }
    std::vector<float> hf(h.size());
    for (size_t i = 0; i < h.size(); ++i) hf[i] = (float)h[i];
    SG_HIP(setup_alloc(&d.p3, h.size() * sizeof(double)));
    if (int rc_ = upload(d.p3, h.data(), h.size() * sizeof(double))) return rc_;
    SG_HIP(setup_alloc(&d.p3f, hf.size() * sizeof(float)));
    if (int rc_ = upload(d.p3f, hf.data(), hf.size() * sizeof(float))) return rc_;
    return SG_OK;
}

static int upload_one(DenseB& d, const std::vector<double>& e) {
    const size_t cnt = e.size();
    std::vector<float> f32(cnt);
    std::vector<uint16_t> hi(cnt), lo(cnt);
    for (size_t i = 0; i < cnt; ++i) {
        f32[i] = (float)e[i];
        hi[i] = host_bf16((float)e[i]);
        lo[i] = host_bf16((float)(e[i] - (double)host_bf16_f(hi[i])));
    }
    SG_HIP(setup_alloc(&d.f64, cnt * sizeof(double)));
    SG_HIP(setup_alloc(&d.f32, cnt * sizeof(float)));
    SG_HIP(setup_alloc(&d.bf_hi, cnt * sizeof(uint16_t)));
    SG_HIP(setup_alloc(&d.bf_lo, cnt * sizeof(uint16_t)));
    if (int rc_ = upload(d.f64, e.data(), cnt * sizeof(double))) return rc_;
    if (int rc_ = upload(d.f32, f32.data(), cnt * sizeof(float))) return rc_;
    if (int rc_ = upload(d.bf_hi, hi.data(), cnt * sizeof(uint16_t))) return rc_;
    if (int rc_ = upload(d.bf_lo, lo.data(), cnt * sizeof(uint16_t))) return rc_;
    return SG_OK;
}

int upload_dense_b(Ctx* c, hipStream_t) {
    const int N = c->n, ld = bexp_ld(N);
    std::vector<cplx> Bf((size_t)N * N), Bi((size_t)N * N);
    for (int x = 0; x < N; ++x)
        for (int a = 0; a < N; ++a) {
            Bf[(size_t)x * N + a] = c->Vt[(size_t)x * N + a];   // forward: B[k=x][n=a] = Ṽ[x][a]
            Bi[(size_t)a * N + x] = c->Vt[(size_t)x * N + a];   // inverse: B[k=a][n=x] = Ṽ[x][a]
        }
    std::vector<double> e;
    expand_bt(N, Bf, e, ld);
    int rc = upload_one(c->fwd, e);
    if (rc) return rc;
    expand_bt(N, Bi, e, ld);
    if ((rc = upload_one(c->inv, e))) return rc;
    if ((rc = upload_planes(c->fwd, N, Bf, ld))) return rc;
    return upload_planes(c->inv, N, Bi, ld);
}

// Tile shapes (see SG_GEMM_NCFG): BM = 32·WM rows; BN = 32·WN real columns for the
// expanded real form (cfg < 5), 32·WN complex columns for the 3M form (cfg >= 5).
static const int kGemmWM[SG_GEMM_NCFG] = {4, 2, 2, 2, 1, 1, 2, 1, 2, 2, 4};
static const int kGemmWN[SG_GEMM_NCFG] = {4, 4, 2, 1, 2, 1, 1, 2, 2, 8, 8};

void gemm_tiles(int cfg, int M, int Nc, int* tiles_m, int* tiles_n) {
    const int bm = 32 * kGemmWM[cfg], bn = 32 * kGemmWN[cfg];
    const int cols = gemm_cfg_3m(cfg) ? Nc / 2 : Nc;   // 3M tiles count complex columns
    *tiles_m = (M + bm - 1) / bm;
    *tiles_n = (cols + bn - 1) / bn;
}

GemmTask make_gemm_task(int precision, const double* A, long long lda, const DenseB& B, int N, double* C,
                        long long ldc, int M, int cfg) {
    GemmTask g{};
    g.A = A;
    g.C = C;
    g.Bt0 = precision == SG_PREC_F64 ? (const void*)B.f64
          : precision == SG_PREC_F32 ? (const void*)B.f32 : (const void*)B.bf_hi;
    g.Bt1 = precision == SG_PREC_BF16X3 ? (const void*)B.bf_lo : nullptr;
    if (gemm_cfg_3m(cfg)) {   // 3M planes, FP64 or FP32
        const size_t plane = (size_t)N * bexp_ld(N);
        g.Bt0 = precision == SG_PREC_F64 ? (const void*)B.p3 : (const void*)B.p3f;
        g.Bt1 = precision == SG_PREC_F64 ? (const void*)(B.p3 + plane) : (const void*)(B.p3f + plane);
    }
    g.lda = 2 * lda;
    g.ldc = 2 * ldc;
    g.ldb = bexp_ld(N);
    g.M = M;
    g.Nc = 2 * N;
    g.Kc = 2 * N;
    gemm_tiles(cfg, M, g.Nc, &g.tiles_m, &g.tiles_n);
    return g;
}

// One transform, with the element types of A and C that g.io names (the FP32 intermediate
// exists only in the reduced-precision forms).
template <int MODE, int WM, int WN, bool M3>
static void launch_single(const GemmTask& g, dim3 grid, hipStream_t st) {
    if constexpr (MODE != MODE_F64) {
        if (g.io == GEMM_IO_C32) {
            if constexpr (M3) hipLaunchKernelGGL((k_gemm3m<MODE, WM, WN, GEMM_IO_C32>), grid, dim3(256), 0, st, g);
            else hipLaunchKernelGGL((k_gemm<MODE, WM, WN, GEMM_IO_C32>), grid, dim3(256), 0, st, g);
            return;
        }
        if (g.io == GEMM_IO_A32) {
            if constexpr (M3) hipLaunchKernelGGL((k_gemm3m<MODE, WM, WN, GEMM_IO_A32>), grid, dim3(256), 0, st, g);
            else hipLaunchKernelGGL((k_gemm<MODE, WM, WN, GEMM_IO_A32>), grid, dim3(256), 0, st, g);
            return;
        }
    }
    if constexpr (M3) hipLaunchKernelGGL((k_gemm3m<MODE, WM, WN, GEMM_IO_F64>), grid, dim3(256), 0, st, g);
    else hipLaunchKernelGGL((k_gemm<MODE, WM, WN, GEMM_IO_F64>), grid, dim3(256), 0, st, g);
}

// Many transforms of one tile shape and one pair of element types (io) in one launch.
template <int MODE, int WM, int WN, bool M3>
static void launch_grouped(int io, dim3 grid, hipStream_t st, const GemmTask* d_tasks, const int* d_start, int ntask,
                           int total) {
#define SG_GROUPED(IO_)                                                                                         \
    do {                                                                                                        \
        if constexpr (M3)                                                                                       \
            hipLaunchKernelGGL((k_gemm3m_grouped<MODE, WM, WN, IO_>), grid, dim3(256), 0, st, d_tasks, d_start,   \
                               ntask, total);                                                                   \
        else                                                                                                    \
            hipLaunchKernelGGL((k_gemm_grouped<MODE, WM, WN, IO_>), grid, dim3(256), 0, st, d_tasks, d_start,     \
                               ntask, total);                                                                   \
    } while (0)
    if constexpr (MODE != MODE_F64) {
        if (io == GEMM_IO_C32) { SG_GROUPED(GEMM_IO_C32); return; }
        if (io == GEMM_IO_A32) { SG_GROUPED(GEMM_IO_A32); return; }
    }
    SG_GROUPED(GEMM_IO_F64);
#undef SG_GROUPED
}

template <int MODE>
static void launch_gemm_cfg(int cfg, const GemmTask& g, const GemmTask* d_tasks, const int* d_start, int ntask,
                            int total, hipStream_t st) {
    const int nt = d_tasks ? total : g.tiles_m * g.tiles_n;
    const dim3 grid(((nt + 7) / 8) * 8), blk(256);
#define SG_GEMM_CFG(C_, WM_, WN_)                                                                          \
    case C_:                                                                                               \
        if (d_tasks) launch_grouped<MODE, WM_, WN_, false>(g.io, grid, st, d_tasks, d_start, ntask, total);  \
        else launch_single<MODE, WM_, WN_, false>(g, grid, st);                                              \
        break;
    switch (cfg) {
        SG_GEMM_CFG(0, 4, 4)
        SG_GEMM_CFG(1, 2, 4)
        SG_GEMM_CFG(2, 2, 2)
        SG_GEMM_CFG(3, 2, 1)
        SG_GEMM_CFG(4, 1, 2)
        default: break;
    }
    if constexpr (MODE != MODE_F64) {   // wide tiles (the FP64 accumulators would not fit)
        switch (cfg) {
            SG_GEMM_CFG(9, 2, 8)
            SG_GEMM_CFG(10, 4, 8)
            default: break;
        }
    }
#undef SG_GEMM_CFG
}

template <int MODE>
static void launch_gemm3m_cfg(int cfg, const GemmTask& g, const GemmTask* d_tasks, const int* d_start, int ntask,
                              int total, hipStream_t st) {
    const int nt = d_tasks ? total : g.tiles_m * g.tiles_n;
    const dim3 grid(((nt + 7) / 8) * 8), blk(256);
#define SG_GEMM3(C_, WM_, WN_)                                                                              \
    case C_:                                                                                                \
        if (d_tasks) launch_grouped<MODE, WM_, WN_, true>(g.io, grid, st, d_tasks, d_start, ntask, total);   \
        else launch_single<MODE, WM_, WN_, true>(g, grid, st);                                               \
        break;
    switch (cfg) {
        SG_GEMM3(5, 1, 1)
        SG_GEMM3(6, 2, 1)
        SG_GEMM3(7, 1, 2)
        SG_GEMM3(8, 2, 2)
        default: break;
    }
#undef SG_GEMM3
}

static int dispatch_gemm(int precision, int cfg, const GemmTask& g, const GemmTask* d_tasks, const int* d_start,
                         int ntask, int total, hipStream_t st) {
    if (!gemm_cfg_valid(cfg, precision)) return fail(SG_EINVAL, "GEMM tile configuration not available in this precision");
    if (gemm_cfg_3m(cfg)) {
        if (precision == SG_PREC_F64) launch_gemm3m_cfg<MODE_F64>(cfg, g, d_tasks, d_start, ntask, total, st);
        else launch_gemm3m_cfg<MODE_F32>(cfg, g, d_tasks, d_start, ntask, total, st);
        SG_HIP(hipGetLastError());
        return SG_OK;
    }
    switch (precision) {
        case SG_PREC_F64: launch_gemm_cfg<MODE_F64>(cfg, g, d_tasks, d_start, ntask, total, st); break;
        case SG_PREC_F32: launch_gemm_cfg<MODE_F32>(cfg, g, d_tasks, d_start, ntask, total, st); break;
        case SG_PREC_BF16X3: launch_gemm_cfg<MODE_BF16X3>(cfg, g, d_tasks, d_start, ntask, total, st); break;
        default: return fail(SG_EINVAL, "unknown precision");
    }
    SG_HIP(hipGetLastError());
    return SG_OK;
}

// Tile shape of an untuned (n, Q, precision), from the autotuner's choices on the
// configurations: the 3M form in FP64 and FP32 (32×32 complex tiles, 64×64 once there are
// more than about eight rounds of 32×32 tiles over the chip), the 64×128 real-form tile in
// BF16x3 (64×256 for n > 384).
int gemm_default_cfg(int N, int M, int precision) {
    if (precision == SG_PREC_BF16X3) return N > 384 ? 9 : 1;
    const long long tiles32 = (long long)((M + 31) / 32) * ((N + 31) / 32);
    return tiles32 > 10240 ? 8 : 5;
}

int gemm_cfg_for(int N, int M, int precision) {
    const int cfg = tune_get(N, M / N, precision);   // the autotuner's choice when tuned
    return gemm_cfg_valid(cfg, precision) ? cfg : gemm_default_cfg(N, M, precision);
}

static int launch_gemm(int precision, const double* A, long long lda, const DenseB& B, int N, double* C,
                       long long ldc, int M, int io, hipStream_t st) {
    const int cfg = gemm_cfg_for(N, M, precision);
    GemmTask g = make_gemm_task(precision, A, lda, B, N, C, ldc, M, cfg);
    g.io = io;
    // algorithmic flops: 8 real flops per complex multiply-add, 6 with the 3M form
    const double cmacs = (double)M * N * N;
    KScope ks(SG_K_GEMM, (gemm_cfg_3m(cfg) ? 6.0 : 8.0) * cmacs, st);
    return dispatch_gemm(precision, cfg, g, nullptr, nullptr, 0, 0, st);
}

int launch_gemm_grouped(int precision, int cfg, int io, const GemmTask* d_tasks, const int* d_start, int ntask,
                        int total, double flops, hipStream_t st) {
    if (ntask <= 0 || total <= 0) return SG_OK;
    if (precision == SG_PREC_F64 && io != GEMM_IO_F64) return fail(SG_EINVAL, "FP64 transforms read and write FP64");
    KScope ks(SG_K_GEMM, flops, st);
    GemmTask g{};
    g.io = io;
    return dispatch_gemm(precision, cfg, g, d_tasks, d_start, ntask, total, st);
}

// Two right-hand sides per thread need whole sets of systems per block (2D, n >= 256/K),
// at least two right-hand sides and segments of at most 8 rows (both in registers).
bool tri_nr_ok(const TriFactors& f, int n, int Q, int dim) {
    return dim == 2 && f.K >= 1 && n >= 256 / f.K && Q >= 2 && f.L <= 8;
}
// In FP32 the rows of two right-hand sides fit in registers up to 16-row segments.
bool tri_nr_ok32(const TriFactors& f, int n, int Q, int dim) {
    return dim == 2 && f.K >= 1 && n >= 256 / f.K && Q >= 2 && f.L <= 16;
}

TriTask make_tri_task(const TriFactors& f, double2* X, int n, int ld, int Q, int dim, int nr) {
    TriTask t{};
    t.X = X;
    t.f = f;
    t.len = n;
    if (dim == 2) {
        t.na = n; t.nq = Q; t.se = ld; t.sa = 1; t.sq = (long long)n * ld; t.fa = 1;
    } else {
        t.na = 1; t.nq = Q; t.se = 1; t.sa = 0; t.sq = n; t.fa = 0;
    }
    t.nblocks = (int)tri_blocks(t.na, t.nq, f.K >= 1 ? f.K : 1, nr);
    return t;
}

int launch_tri_grouped(const TriTask* d_tasks, const int* d_start, int ntask, int total, int max_seg, int nr,
                       bool f32, double bytes, hipStream_t st) {
    if (ntask <= 0 || total <= 0) return SG_OK;
    if (max_seg > 32) return fail(SG_EINVAL, "grid too large for the grouped tridiagonal sweep");
    if (nr == 2 && max_seg > (f32 ? 16 : 8))
        return fail(SG_EINVAL, "two right-hand sides per thread need segments of <= 8 rows (16 in FP32)");
    KScope ks(SG_K_TRI, bytes, st);
    const dim3 grid((unsigned)((total + 7) / 8 * 8));
#define SG_TRIG(SEGL_, NR_, T2_) \
    hipLaunchKernelGGL((k_tri_seg_grouped<SEGL_, NR_, T2_>), grid, dim3(256), 0, st, d_tasks, d_start, ntask, total)
    if (f32) {
        if (nr == 2) {
            if (max_seg <= 8) SG_TRIG(8, 2, float2);
            else SG_TRIG(16, 2, float2);
        } else if (max_seg <= 8) SG_TRIG(8, 1, float2);
        else if (max_seg <= 16) SG_TRIG(16, 1, float2);
        else SG_TRIG(32, 1, float2);
    } else if (nr == 2) SG_TRIG(8, 2, double2);
    else if (max_seg <= 8) SG_TRIG(8, 1, double2);
    else if (max_seg <= 16) SG_TRIG(16, 1, double2);
    else SG_TRIG(32, 1, double2);
#undef SG_TRIG
    SG_HIP(hipGetLastError());
    return SG_OK;
}

// X holds double2 elements, or float2 ones when f32 (the FP32 intermediate of the
// reduced-precision forms, which only the segmented kernel serves).
static int launch_tri(const TriFactors& f, void* X, bool f32, int n, int ld, int Q, int dim, hipStream_t st) {
    int na, nq, fa;
    long long se, sa, sq;
    if (dim == 2) {
        na = n; nq = Q; se = ld; sa = 1; sq = (long long)n * ld; fa = 1;
    } else {
        na = 1; nq = Q; se = 1; sa = 0; sq = n; fa = 0;
    }
    const long long nth = (long long)na * nq;
    const int blk = 64;
    // algorithmic: every element read and written once, factors read once
    KScope ks(SG_K_TRI, (f32 ? 16.0 : 32.0) * na * (double)nq * n + 65.0 * f.nsys * (double)n, st);
    if (f.L <= 32 && f.K >= 1) {
        // two right-hand sides per thread where the blocks hold whole sets of systems and the
        // segments are short enough for both to stay in registers (FP64, 8 rows: 166
        // registers; 16 rows would spill)
        const int nr = (f32 ? tri_nr_ok32(f, n, Q, dim) : tri_nr_ok(f, n, Q, dim)) ? 2 : 1;
        const long long total = tri_blocks(na, nq, f.K, nr);
        if (total > INT32_MAX - 8) return fail(SG_EINVAL, "grid too large for the tridiagonal sweep");
        const dim3 grid((unsigned)((total + 7) / 8 * 8));
#define SG_TRI(SEGL_, NR_, T2_)                                                                                    \
    hipLaunchKernelGGL((k_tri_seg<SEGL_, NR_, T2_>), grid, dim3(256), 0, st, static_cast<T2_*>(X), f, n, na, nq, se, \
                       sa, sq, fa, (int)total)
        if (f32) {
            if (nr == 2) {
                if (f.L <= 8) SG_TRI(8, 2, float2);
                else SG_TRI(16, 2, float2);
            } else {
                if (f.L <= 8) SG_TRI(8, 1, float2);
                else if (f.L <= 16) SG_TRI(16, 1, float2);
                else SG_TRI(32, 1, float2);
            }
        } else if (nr == 2) {
            SG_TRI(8, 2, double2);
        } else {
            if (f.L <= 8) SG_TRI(8, 1, double2);
            else if (f.L <= 16) SG_TRI(16, 1, double2);
            else SG_TRI(32, 1, double2);
        }
#undef SG_TRI
        SG_HIP(hipGetLastError());
        return SG_OK;
    }
    if (f32) return fail(SG_EINVAL, "internal: the FP32 sweep needs the segmented factors");
    hipLaunchKernelGGL(k_tri, dim3((unsigned)((nth + blk - 1) / blk)), dim3(blk), 0, st, static_cast<double2*>(X), f,
                       n, na, nq, se, sa, sq, fa);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int launch_precond(Ctx* c, int pc, int precision, const double2* r, double2* z, hipStream_t st) {
    if (pc == SG_PC_NONE) {
        if (r != z) SG_HIP(hipMemcpyAsync(z, r, (size_t)c->nvec * sizeof(double2), hipMemcpyDeviceToDevice, st));
        return SG_OK;
    }
    if (pc != SG_PC_MEAN && pc != SG_PC_CSL_MEAN) return fail(SG_EINVAL, "sg_precond: unknown preconditioner");
    if (precision < SG_PREC_F64 || precision > SG_PREC_BF16X3) return fail(SG_EINVAL, "sg_precond: unknown precision");
    if (c->vmean) {
        if (precision != SG_PREC_F64)
            return fail(SG_EINVAL, "sg_precond: a spatially varying mean is solved in FP64 only");
        return launch_line(c, pc, r, z, st);
    }
    const TriFactors& f = c->tri[pc == SG_PC_MEAN ? 0 : 1];
    const int n = c->n;
    if (c->dim == 1) {
        if (r != z) SG_HIP(hipMemcpyAsync(z, r, (size_t)c->nvec * sizeof(double2), hipMemcpyDeviceToDevice, st));
        return launch_tri(f, z, false, n, n, c->Q, 1, st);
    }
    const int M = c->Q * n;
    double2* t = c->d_tmp_pc;
    // The reduced-precision forms keep the intermediate W (transform output, sweep, transform
    // input) in FP32: the transforms round it to FP32 anyway, and half the bytes move.
    const bool t32 = precision != SG_PREC_F64 && f.L <= 32 && f.K >= 1;
    int rc = launch_gemm(precision, reinterpret_cast<const double*>(r), n, c->fwd, n, reinterpret_cast<double*>(t),
                         c->tld, M, t32 ? GEMM_IO_C32 : GEMM_IO_F64, st);
    if (rc) return rc;
    rc = launch_tri(f, t, t32, n, c->tld, c->Q, 2, st);
    if (rc) return rc;
    return launch_gemm(precision, reinterpret_cast<const double*>(t), c->tld, c->inv, n, reinterpret_cast<double*>(z),
                       n, M, t32 ? GEMM_IO_A32 : GEMM_IO_F64, st);
}

}  // namespace sgi
