// Kernels of the learned correction network (a 3-level convolutional U-Net applied after
// the mean-value block solve inside flexible GMRES): BF16 tensors, FP32 accumulation on
// the matrix cores, FP32 master weights and gradients.
//
// Tensors are NHWC ([image][row][column][channel], channels fastest) with the channel
// count padded to a multiple of 32, so that one 16-byte load gives a lane the eight
// consecutive channels an MFMA operand needs.
//
//  conv      3×3 (or 1×1) convolution as an implicit GEMM D[co][pixel] on
//            v_mfma_f32_16x16x32_bf16: A = weights [co][tap][ci], B = input pixels
//            [pixel][ci], both read straight from global memory; bias, ReLU and the
//            backward ReLU mask are applied in the epilogue.  The input gradient of a
//            convolution is the same kernel with the tap-flipped, transposed weights.
//  wgrad     dW[co][tap][ci] = Σ_pixels dZ[pixel][co] X[pixel + tap][ci], split over pixel
//            chunks; tiles are transposed through LDS into the MFMA operand layout; the
//            chunk partials are summed in a fixed order (deterministic).
//  small     pooling, upsampling + concatenation, their adjoints, packing of SG vectors,
//            loss, Adam, weight conversion.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "net_internal.h"

namespace sgi {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ bf8 load8(const uint16_t* p) { return *reinterpret_cast<const bf8*>(p); }
__device__ __forceinline__ bf8 zero8() { return __builtin_bit_cast(bf8, make_uint4(0, 0, 0, 0)); }

// Y[b][p][co] for a block of 128 pixels (4 waves × 2 fragments of 16) and 16·NC channels.
template <int NC, int KS, bool RELU, bool OUTF32, bool MASK>
__global__ __launch_bounds__(256) void k_conv(const uint16_t* __restrict__ X, int Cin, const uint16_t* __restrict__ Wt,
                                              const float* __restrict__ bias, void* __restrict__ Yv, int Cout,
                                              const uint16_t* __restrict__ mask, int H, int W) {
    constexpr int KK = KS * KS;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int HW = H * W;
    const long long img = blockIdx.z;
    const int co0 = blockIdx.y * (16 * NC);
    const int pbase = blockIdx.x * 128 + wv * 32;
    const uint16_t* __restrict__ Xi = X + img * HW * Cin;
    int py[2], px[2];
    bool pv[2];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        const int p = pbase + f * 16 + l16;
        pv[f] = p < HW;
        py[f] = pv[f] ? p / W : 0;
        px[f] = pv[f] ? p - py[f] * W : 0;
    }
    f4 acc[NC][2];
#pragma unroll
    for (int i = 0; i < NC; ++i)
#pragma unroll
        for (int f = 0; f < 2; ++f) acc[i][f] = f4{0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < KK; ++t) {
        const int dy = KS == 3 ? t / 3 - 1 : 0, dx = KS == 3 ? t % 3 - 1 : 0;
        const uint16_t* src[2];
        bool ok[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            const int yy = py[f] + dy, xx = px[f] + dx;
            ok[f] = pv[f] && yy >= 0 && yy < H && xx >= 0 && xx < W;
            src[f] = Xi + (long long)(ok[f] ? yy * W + xx : 0) * Cin + lq * 8;
        }
        const uint16_t* wsrc = Wt + ((long long)(co0 + l16) * KK + t) * Cin + lq * 8;
        for (int c0 = 0; c0 < Cin; c0 += 32) {
            bf8 bv[2], av[NC];
#pragma unroll
            for (int f = 0; f < 2; ++f) bv[f] = ok[f] ? load8(src[f] + c0) : zero8();
#pragma unroll
            for (int i = 0; i < NC; ++i) av[i] = load8(wsrc + (long long)i * 16 * KK * Cin + c0);
#pragma unroll
            for (int i = 0; i < NC; ++i)
#pragma unroll
                for (int f = 0; f < 2; ++f)
                    acc[i][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[f], acc[i][f], 0, 0, 0);
        }
    }
    // lane (lq, l16) holds D[co = co0 + 16i + 4lq + v][pixel = pbase + 16f + l16]
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        const int p = pbase + f * 16 + l16;
        if (p >= HW) continue;
        const long long o = (img * HW + p) * Cout;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const int co = co0 + i * 16 + 4 * lq;
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                float a = acc[i][f][u] + (bias ? bias[co + u] : 0.f);
                if (RELU) a = fmaxf(a, 0.f);
                if (MASK && !(bf2f(mask[o + co + u]) > 0.f)) a = 0.f;
                v[u] = a;
            }
            if constexpr (OUTF32) {
                *reinterpret_cast<float4*>(reinterpret_cast<float*>(Yv) + o + co) = make_float4(v[0], v[1], v[2], v[3]);
            } else {
                const uint32_t lo = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
                const uint32_t hi = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
                *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(Yv) + o + co) = make_uint2(lo, hi);
            }
        }
    }
}

// 3×3 convolution with the input tile in LDS.  The block's PIX = 64·NF pixels (row-major
// from P0; 4 waves × NF fragments of 16) with their one-pixel halo are staged once per
// 32-channel chunk: rows r0-1 .. r1+1 and, when the pixels lie in one row, the columns
// x0-1 .. x0+PIX, else whole rows -1 .. W (out of the image: zeros).  The nine taps then
// read their operands from LDS instead of re-reading the input from the caches nine times.
// NF and the output channels per block (16·NC) are chosen per layer by the launcher: the
// coarse tiles (NF = 2) for the large layers, the fine ones where the coarse grid would
// leave CUs idle (the 128² and 64² levels at batch 1).  (Four fragments per wave measured
// slower: 50 KB of LDS leaves three blocks per CU.)  Output as in k_conv.
constexpr int CONV_TILE_PIX = 640;   // LDS pixels per chunk (40 KB)

__host__ __device__ inline void conv_tile_shape(int P0, int pix, int H, int W, int* r0, int* rows, int* x0, int* cols) {
    const int HW = H * W;
    const int plast = (P0 + pix - 1 < HW ? P0 + pix - 1 : HW - 1);
    *r0 = P0 / W;
    const int r1 = plast / W;
    *rows = r1 - *r0 + 3;
    if (r1 == *r0) {
        *x0 = P0 % W - 1;
        *cols = (plast % W) - (P0 % W) + 3;
    } else {
        *x0 = -1;
        *cols = W + 2;
    }
}

template <int NC, int NF, bool RELU, bool OUTF32, bool MASK>
__global__ __launch_bounds__(256) void k_conv3l(const uint16_t* __restrict__ X, int Cin, const uint16_t* __restrict__ Wt,
                                                const float* __restrict__ bias, void* __restrict__ Yv, int Cout,
                                                const uint16_t* __restrict__ mask, int H, int W) {
    constexpr int KK = 9;
    __shared__ uint4 tile[CONV_TILE_PIX * 4];   // [pixel][4 groups of 8 channels]
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int HW = H * W;
    const long long img = blockIdx.z;
    const int co0 = blockIdx.y * (16 * NC);
    constexpr int PIX = 64 * NF;
    const int P0 = blockIdx.x * PIX;
    const int pbase = P0 + wv * 16 * NF;
    const uint16_t* __restrict__ Xi = X + img * HW * Cin;
    int r0, rows, x0, cols;
    conv_tile_shape(P0, PIX, H, W, &r0, &rows, &x0, &cols);
    const int npix = rows * cols;   // <= CONV_TILE_PIX (checked by the launcher)
    int lp[NF];
    bool pv[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const int p = pbase + f * 16 + l16;
        pv[f] = p < HW;
        const int py = pv[f] ? p / W : r0, px = pv[f] ? p - (p / W) * W : x0 + 1;
        lp[f] = (py - r0 + 1) * cols + (px - x0);   // tile index of the pixel itself
    }
    f4 acc[NC][NF];
#pragma unroll
    for (int i = 0; i < NC; ++i)
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[i][f] = f4{0.f, 0.f, 0.f, 0.f};
    // with 32 output channels per block the chunk's weight fragments of all nine taps fit in
    // registers: they are loaded before the input tile is staged, so that their latency
    // overlaps the staging instead of stalling every tap
    constexpr bool PRE = NC <= 2;
    for (int c0 = 0; c0 < Cin; c0 += 32) {
        __syncthreads();   // the previous chunk's reads are done
        bf8 wr[PRE ? KK : 1][NC];
        if constexpr (PRE) {
            const uint16_t* wsrc0 = Wt + (long long)(co0 + l16) * KK * Cin + c0 + lq * 8;
#pragma unroll
            for (int t = 0; t < KK; ++t)
#pragma unroll
                for (int i = 0; i < NC; ++i) wr[t][i] = load8(wsrc0 + (long long)t * Cin + (long long)i * 16 * KK * Cin);
        }
        for (int e = threadIdx.x; e < npix * 4; e += 256) {
            const int q = e >> 2, part = e & 3;
            const int rr = q / cols, cc = q - rr * cols;
            const int y = r0 - 1 + rr, x = x0 + cc;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (y >= 0 && y < H && x >= 0 && x < W)
                v = *reinterpret_cast<const uint4*>(Xi + (long long)(y * W + x) * Cin + c0 + part * 8);
            tile[e] = v;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < KK; ++t) {
            const int dy = t / 3 - 1, dx = t % 3 - 1;
            bf8 bv[NF], av[NC];
#pragma unroll
            for (int f = 0; f < NF; ++f)
                bv[f] = pv[f] ? __builtin_bit_cast(bf8, tile[(lp[f] + dy * cols + dx) * 4 + lq]) : zero8();
            if constexpr (PRE) {
#pragma unroll
                for (int i = 0; i < NC; ++i) av[i] = wr[t][i];
            } else {
                const uint16_t* wsrc = Wt + ((long long)(co0 + l16) * KK + t) * Cin + c0 + lq * 8;
#pragma unroll
                for (int i = 0; i < NC; ++i) av[i] = load8(wsrc + (long long)i * 16 * KK * Cin);
            }
#pragma unroll
            for (int i = 0; i < NC; ++i)
#pragma unroll
                for (int f = 0; f < NF; ++f)
                    acc[i][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[f], acc[i][f], 0, 0, 0);
        }
    }
    // lane (lq, l16) holds D[co = co0 + 16i + 4lq + v][pixel = pbase + 16f + l16]
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const int p = pbase + f * 16 + l16;
        if (p >= HW) continue;
        const long long o = (img * HW + p) * Cout;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const int co = co0 + i * 16 + 4 * lq;
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                float a = acc[i][f][u] + (bias ? bias[co + u] : 0.f);
                if (RELU) a = fmaxf(a, 0.f);
                if (MASK && !(bf2f(mask[o + co + u]) > 0.f)) a = 0.f;
                v[u] = a;
            }
            if constexpr (OUTF32) {
                *reinterpret_cast<float4*>(reinterpret_cast<float*>(Yv) + o + co) = make_float4(v[0], v[1], v[2], v[3]);
            } else {
                const uint32_t lo = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
                const uint32_t hi = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
                *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(Yv) + o + co) = make_uint2(lo, hi);
            }
        }
    }
}

// Weight gradient partials: block (ci-block of 32 × tap, co-block of 32, image × pixel
// chunk) accumulates D[co][ci] over CHUNK pixels in stages of 128; wave w takes pixels
// [32w, 32w+32) of every stage; the four waves are summed through LDS at the end.
constexpr int WG_STAGE = 128, WG_CHUNK = 1024, WG_LD = WG_STAGE + 8;

template <int KS>
__global__ __launch_bounds__(256) void k_wgrad(const uint16_t* __restrict__ dZ, int Cout, const uint16_t* __restrict__ X,
                                               int Cin, int H, int W, int nchunk, float* __restrict__ partial) {
    constexpr int KK = KS * KS;
    __shared__ uint16_t sA[32 * WG_LD];   // dZ tile, transposed: [co][pixel]
    __shared__ uint16_t sB[32 * WG_LD];   // shifted X tile, transposed: [ci][pixel]
    __shared__ float red[4][32 * 32];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int cib = blockIdx.x / KK, t = blockIdx.x % KK;
    const int dy = KS == 3 ? t / 3 - 1 : 0, dx = KS == 3 ? t % 3 - 1 : 0;
    const int ci0 = cib * 32, co0 = blockIdx.y * 32;
    const long long img = blockIdx.z / nchunk;
    const int chunk = blockIdx.z % nchunk;
    const int HW = H * W;
    const uint16_t* __restrict__ dZi = dZ + img * HW * Cout;
    const uint16_t* __restrict__ Xi = X + img * HW * Cin;
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    const int pend = min(HW, (chunk + 1) * WG_CHUNK);
    for (int s0 = chunk * WG_CHUNK; s0 < pend; s0 += WG_STAGE) {
        // 128 pixels × 4 groups of 8 channels, for each of the two tiles: 2 loads per thread
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int idx = r * 256 + threadIdx.x, pl = idx >> 2, g = idx & 3;
            const int p = s0 + pl;
            uint4 za = make_uint4(0, 0, 0, 0), xb = make_uint4(0, 0, 0, 0);
            if (p < pend) {
                za = *reinterpret_cast<const uint4*>(dZi + (long long)p * Cout + co0 + g * 8);
                const int yy = p / W + dy, xx = p % W + dx;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                    xb = *reinterpret_cast<const uint4*>(Xi + (long long)(yy * W + xx) * Cin + ci0 + g * 8);
            }
            const uint16_t* a16 = reinterpret_cast<const uint16_t*>(&za);
            const uint16_t* b16 = reinterpret_cast<const uint16_t*>(&xb);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                sA[(g * 8 + u) * WG_LD + pl] = a16[u];
                sB[(g * 8 + u) * WG_LD + pl] = b16[u];
            }
        }
        __syncthreads();
        bf8 av[2], bv[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            av[i] = load8(&sA[(i * 16 + l16) * WG_LD + wv * 32 + lq * 8]);
            bv[i] = load8(&sB[(i * 16 + l16) * WG_LD + wv * 32 + lq * 8]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // lane holds D[co = 16i + 4lq + v][ci = 16j + l16]
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int u = 0; u < 4; ++u) red[wv][(i * 16 + 4 * lq + u) * 32 + j * 16 + l16] = acc[i][j][u];
    __syncthreads();
    float* out = partial + (long long)blockIdx.z * Cout * KK * Cin;
    for (int e = threadIdx.x; e < 32 * 32; e += 256) {
        const float v = red[0][e] + red[1][e] + red[2][e] + red[3][e];
        const int co = co0 + e / 32, ci = ci0 + e % 32;
        out[((long long)co * KK + t) * Cin + ci] = v;
    }
}

// Sum of the nz partials into the flat gradient (unpadded [co][kh][kw][ci] layout).
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ partial, int nz, int Cout, int KK,
                                                      int Cin, int co_real, int ci_real, float* __restrict__ g) {
    const long long n = (long long)co_real * KK * ci_real;
    const long long stride = (long long)Cout * KK * Cin;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const int ci = (int)(e % ci_real);
        const long long r = e / ci_real;
        const int t = (int)(r % KK), co = (int)(r / KK);
        const long long src = ((long long)co * KK + t) * Cin + ci;
        float s = 0.f;
        for (int z = 0; z < nz; ++z) s += partial[z * stride + src];
        g[e] = s;
    }
}

// Bias gradient: partial[block][co] = Σ over the block's pixels of dZ[pixel][co].  Thread t
// sums channels 8·(t mod G) .. +7 (one 16-byte load, G = C/8 groups per pixel) over the
// pixels t/G, t/G + 256/G, ... of the block; the 256/G row sums of a channel are then added
// in a fixed order (deterministic).
constexpr int COLSUM_PER = 256;   // pixels per block
__global__ __launch_bounds__(256) void k_colsum(const uint16_t* __restrict__ dZ, long long npix, int C, int per_block,
                                                float* __restrict__ partial) {
    __shared__ float red[256 * 8];
    const int G = C / 8, rows = 256 / G, lanes = rows * G;
    const int t = threadIdx.x, g = t % G;
    float s[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] = 0.f;
    if (t < lanes) {
        const long long p0 = (long long)blockIdx.x * per_block;
        const long long p1 = min(npix, p0 + per_block);
        for (long long p = p0 + t / G; p < p1; p += rows) {
            const uint4 v = *reinterpret_cast<const uint4*>(dZ + p * C + 8 * g);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s[2 * k] += bf2f((uint16_t)(w[k] & 0xffffu));
                s[2 * k + 1] += bf2f((uint16_t)(w[k] >> 16));
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) red[t * 8 + k] = s[k];
    __syncthreads();
    for (int c = t; c < C; c += 256) {
        float u = 0.f;
        for (int r = 0; r < rows; ++r) u += red[(r * G + c / 8) * 8 + c % 8];
        partial[(long long)blockIdx.x * C + c] = u;
    }
}

// g[c] = Σ_b partial[b][c]: one block per channel, strided partial sums per thread, then a
// fixed-order tree in LDS (deterministic).
__global__ __launch_bounds__(256) void k_colsum_reduce(const float* __restrict__ partial, int nb, int C, int c_real,
                                                       float* __restrict__ g) {
    __shared__ float red[256];
    const int c = blockIdx.x;
    float s = 0.f;
    for (int b = threadIdx.x; b < nb; b += 256) s += partial[(long long)b * C + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0 && c < c_real) g[c] = red[0];
}

// 2×2 average pooling: out[b][y][x][c] = mean of in[b][2y+i][2x+j][c].
__global__ __launch_bounds__(256) void k_pool(const uint16_t* __restrict__ in, uint16_t* __restrict__ out, int Hl, int Wl,
                                              int C, long long n) {
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const int c = (int)(e % C);
        const long long r = e / C;
        const int x = (int)(r % Wl);
        const long long r2 = r / Wl;
        const int y = (int)(r2 % Hl);
        const long long b = r2 / Hl;
        const int Wh = 2 * Wl;
        const long long base = ((b * 2 * Hl + 2 * y) * Wh + 2 * x) * C + c;
        const float s = bf2f(in[base]) + bf2f(in[base + C]) + bf2f(in[base + (long long)Wh * C]) +
                        bf2f(in[base + (long long)Wh * C + C]);
        out[e] = f2bf(0.25f * s);
    }
}

// out[b][y][x][0:Cu] = U[b][y/2][x/2][:], out[..][Cu:Cu+Cs] = S[b][y][x][:]
__global__ __launch_bounds__(256) void k_up_concat(const uint16_t* __restrict__ U, int Cu, const uint16_t* __restrict__ S,
                                                   int Cs, uint16_t* __restrict__ out, int H, int W, long long n) {
    const int C = Cu + Cs;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const int c = (int)(e % C);
        const long long pix = e / C;
        const int x = (int)(pix % W);
        const long long r = pix / W;
        const int y = (int)(r % H);
        const long long b = r / H;
        if (c < Cu) out[e] = U[((b * (H / 2) + y / 2) * (W / 2) + x / 2) * Cu + c];
        else out[e] = S[pix * Cs + (c - Cu)];
    }
}

// Adjoint of up_concat for its first Cu channels, times the ReLU mask of the
// low-resolution tensor: d[b][y][x][c] = mask>0 ? Σ_{i,j} dC[b][2y+i][2x+j][c] : 0.
__global__ __launch_bounds__(256) void k_up_bwd(const uint16_t* __restrict__ dC, int C, int Cu,
                                                const uint16_t* __restrict__ mask, uint16_t* __restrict__ out, int Hl,
                                                int Wl, long long n) {
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const int c = (int)(e % Cu);
        const long long r = e / Cu;
        const int x = (int)(r % Wl);
        const long long r2 = r / Wl;
        const int y = (int)(r2 % Hl);
        const long long b = r2 / Hl;
        const int Wh = 2 * Wl;
        const long long base = ((b * 2 * Hl + 2 * y) * Wh + 2 * x) * C + c;
        const float s = bf2f(dC[base]) + bf2f(dC[base + C]) + bf2f(dC[base + (long long)Wh * C]) +
                        bf2f(dC[base + (long long)Wh * C + C]);
        out[e] = bf2f(mask[e]) > 0.f ? f2bf(s) : (uint16_t)0;
    }
}

// Gradient of a skip tensor: d[b][y][x][c] = mask>0 ? dC[..][Cu + c] + dP[b][y/2][x/2][c] / 4 : 0.
__global__ __launch_bounds__(256) void k_skip_bwd(const uint16_t* __restrict__ dC, int Ccat, int Cu,
                                                  const uint16_t* __restrict__ dP, const uint16_t* __restrict__ mask,
                                                  uint16_t* __restrict__ out, int H, int W, int C, long long n) {
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const int c = (int)(e % C);
        const long long pix = e / C;
        const int x = (int)(pix % W);
        const long long r = pix / W;
        const int y = (int)(r % H);
        const long long b = r / H;
        const float s = bf2f(dC[pix * Ccat + Cu + c]) + 0.25f * bf2f(dP[((b * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c]);
        out[e] = bf2f(mask[e]) > 0.f ? f2bf(s) : (uint16_t)0;
    }
}

// Input tensor of a residual r ([Q][n][n] complex): channels (2q, 2q+1) = (Re, Im) r_q ·
// sqrt(Q n²)/||r||, then k_0/k̄ (= 1) and k_l/k̄; zero in the padding.
__global__ __launch_bounds__(256) void k_pack(const double2* __restrict__ r, const double2* __restrict__ rnorm, int Q,
                                              int n, int H, const double* __restrict__ kf, int s, double kbar, int Cp,
                                              uint16_t* __restrict__ out) {
    const long long np = (long long)H * H;
    const double sc = sqrt((double)Q * n * n) / rnorm->x;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < np * Cp; e += (long long)gridDim.x * 256) {
        const int c = (int)(e % Cp);
        const long long p = e / Cp;
        const int x = (int)(p % H), y = (int)(p / H);
        float v = 0.f;
        if (x < n && y < n) {
            const long long g = (long long)y * n + x;
            if (c < 2 * Q) {
                const double2 z = r[(long long)(c >> 1) * n * n + g];
                v = (float)(((c & 1) ? z.y : z.x) * sc);
            } else if (c == 2 * Q) {
                v = 1.f;
            } else if (c <= 2 * Q + s) {
                v = (float)(kf[(long long)(c - 2 * Q - 1) * n * n + g] / kbar);
            }
        }
        out[e] = f2bf(v);
    }
}

// z += ||z0|| / sqrt(Q n²) · (y[2q] + i y[2q+1]) on the grid (y: [H][H][Cp] FP32).
__global__ __launch_bounds__(256) void k_unpack_add(const float* __restrict__ y, int Cp, const double2* __restrict__ znorm,
                                                    int Q, int n, int H, double2* __restrict__ z) {
    const long long N = (long long)Q * n * n;
    const double sc = znorm->x / sqrt((double)Q * n * n);
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < N; e += (long long)gridDim.x * 256) {
        const int q = (int)(e / ((long long)n * n));
        const long long g = e % ((long long)n * n);
        const int y0 = (int)(g / n), x0 = (int)(g % n);
        const float* yp = y + ((long long)y0 * H + x0) * Cp + 2 * q;
        double2 v = z[e];
        v.x += sc * yp[0];
        v.y += sc * yp[1];
        z[e] = v;
    }
}

// Target tensor of a correction c in units of ||z0|| / sqrt(Q n²) (FP32, zero padding).
__global__ __launch_bounds__(256) void k_pack_target(const double2* __restrict__ c, const double2* __restrict__ znorm,
                                                     int Q, int n, int H, int Cp, float* __restrict__ out) {
    const long long np = (long long)H * H;
    const double sc = sqrt((double)Q * n * n) / znorm->x;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < np * Cp; e += (long long)gridDim.x * 256) {
        const int ch = (int)(e % Cp);
        const long long p = e / Cp;
        const int x = (int)(p % H), y = (int)(p / H);
        float v = 0.f;
        if (x < n && y < n && ch < 2 * Q) {
            const double2 zz = c[(long long)(ch >> 1) * n * n + (long long)y * n + x];
            v = (float)(((ch & 1) ? zz.y : zz.x) * sc);
        }
        out[e] = v;
    }
}

// FP32 NHWC (unpadded channels) → BF16 NHWC (padded channels)
__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ in, int C, uint16_t* __restrict__ out, int Cp,
                                                 long long npix) {
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < npix * Cp; e += (long long)gridDim.x * 256) {
        const int c = (int)(e % Cp);
        const long long p = e / Cp;
        out[e] = c < C ? f2bf(in[p * C + c]) : (uint16_t)0;
    }
}

// FP32 NHWC (unpadded) → FP32 NHWC (padded)
__global__ __launch_bounds__(256) void k_pad_f32(const float* __restrict__ in, int C, float* __restrict__ out, int Cp,
                                                 long long npix) {
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < npix * Cp; e += (long long)gridDim.x * 256) {
        const int c = (int)(e % Cp);
        const long long p = e / Cp;
        out[e] = c < C ? in[p * C + c] : 0.f;
    }
}

__global__ __launch_bounds__(256) void k_unpad_f32(const float* __restrict__ in, int Cp, float* __restrict__ out, int C,
                                                   long long npix) {
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < npix * C; e += (long long)gridDim.x * 256) {
        const int c = (int)(e % C);
        const long long p = e / C;
        out[e] = in[p * Cp + c];
    }
}

// Mean squared error over the first C of Cp channels: dY = 2 (y - t) / count (BF16),
// partial[block] = Σ (y - t)².
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ t, long long npix, int Cp,
                                             int C, double inv_count, uint16_t* __restrict__ dy, float* __restrict__ partial) {
    __shared__ float red[256];
    float s = 0.f;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < npix * Cp; e += (long long)gridDim.x * 256) {
        const int c = (int)(e % Cp);
        float g = 0.f;
        if (c < C) {
            const float d = y[e] - t[e];
            s += d * d;
            g = (float)(2.0 * inv_count) * d;
        }
        dy[e] = f2bf(g);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Adam (Kingma & Ba): bias-corrected moments, FP32 state.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, long long n, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const float ge = g[e];
        const float me = b1 * m[e] + (1.f - b1) * ge;
        const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
        m[e] = me;
        v[e] = ve;
        th[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
    }
}

// One layer's master weights (flat [co][kh][kw][ci] + bias) → padded BF16 forward weights
// [Cout_p][KK][Cin_p], tap-flipped transposed weights [Cin_p][KK][Cout_p] and FP32 bias.
__global__ __launch_bounds__(256) void k_weights(const float* __restrict__ th, int co_real, int ci_real, int KK, int Coutp,
                                                 int Cinp, uint16_t* __restrict__ wf, uint16_t* __restrict__ wb,
                                                 float* __restrict__ bias) {
    const long long n = (long long)Coutp * KK * Cinp;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const int ci = (int)(e % Cinp);
        const long long r = e / Cinp;
        const int t = (int)(r % KK), co = (int)(r / KK);
        float w = 0.f;
        if (co < co_real && ci < ci_real) w = th[((long long)co * KK + t) * ci_real + ci];
        const uint16_t b = f2bf(w);
        wf[e] = b;
        wb[((long long)ci * KK + (KK - 1 - t)) * Coutp + co] = b;
        if (t == 0 && ci == 0) bias[co] = co < co_real ? th[(long long)co_real * KK * ci_real + co] : 0.f;
    }
}

inline unsigned grid_of(long long n) {
    long long b = (n + 255) / 256;
    if (b > 16384) b = 16384;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

int net_conv(const uint16_t* X, int Cin, const uint16_t* W, const float* bias, void* Y, int Cout, bool relu, bool out_f32,
             const uint16_t* mask, int H, int Wd, int batch, int ks, hipStream_t st) {
    if (Cin % 32 || Cout % 32) return fail(SG_EINVAL, "net: channel counts must be multiples of 32");
    if (out_f32 && (relu || mask)) return fail(SG_EINVAL, "net: FP32 output is for the linear head only");
    int nc = Cout % 64 == 0 ? 4 : (Cout % 96 == 0 ? 6 : 2);
    if (Cout == 32) nc = 2;
    const dim3 grid((unsigned)((H * Wd + 127) / 128), (unsigned)(Cout / (16 * nc)), (unsigned)batch), blk(256);
    // 3×3 LDS kernel: 128 pixels and 16·nc channels per block, or 64 pixels and 32 channels
    // where that grid would have fewer than four blocks per CU
    auto nblk3 = [&](int c, int f) {
        return (long long)((H * Wd + 64 * f - 1) / (64 * f)) * (Cout / (16 * c)) * batch;
    };
    int nf = 2, nc3 = nc;
    if (nblk3(nc3, nf) < 1024) {
        nf = 1;
        nc3 = 2;
    }
    const int pix = 64 * nf;
    KScope ks_(SG_K_NET, 2.0 * H * Wd * (double)batch * Cout * Cin * ks * ks, st);
#define SG_CONV(NC_, KS_, R_, F_, M_) \
    hipLaunchKernelGGL((k_conv<NC_, KS_, R_, F_, M_>), grid, blk, 0, st, X, Cin, W, bias, Y, Cout, mask, H, Wd)
#define SG_CONV_NC(KS_, R_, F_, M_)                  \
    do {                                             \
        if (nc == 2) SG_CONV(2, KS_, R_, F_, M_);    \
        else if (nc == 4) SG_CONV(4, KS_, R_, F_, M_); \
        else SG_CONV(6, KS_, R_, F_, M_);            \
    } while (0)
    // the LDS-tiled 3×3 kernel when every block's halo tile fits (the tile is largest for
    // the blocks whose pixels span the most rows, at most ceil((pix-1)/W)+1 of them; with W
    // a multiple of pix every block lies in one row)
    const int max_rows = (pix - 1 + Wd - 1) / Wd + 1 + 2;
    const bool lds_fits = (long long)max_rows * (Wd + 2) <= CONV_TILE_PIX ||
                          (Wd % pix == 0 && 3 * (pix + 2) <= CONV_TILE_PIX);
    const dim3 gridl((unsigned)((H * Wd + pix - 1) / pix), (unsigned)(Cout / (16 * nc3)), grid.z);
#define SG_CONVL(NC_, NF_, R_, F_, M_) \
    hipLaunchKernelGGL((k_conv3l<NC_, NF_, R_, F_, M_>), gridl, blk, 0, st, X, Cin, W, bias, Y, Cout, mask, H, Wd)
#define SG_CONVL_NC(R_, F_, M_)                        \
    do {                                               \
        if (nf == 1) SG_CONVL(2, 1, R_, F_, M_);       \
        else if (nc3 == 2) SG_CONVL(2, 2, R_, F_, M_); \
        else if (nc3 == 4) SG_CONVL(4, 2, R_, F_, M_); \
        else SG_CONVL(6, 2, R_, F_, M_);               \
    } while (0)
    if (ks == 3 && lds_fits) {
        if (out_f32) SG_CONVL_NC(false, true, false);
        else if (relu) SG_CONVL_NC(true, false, false);
        else if (mask) SG_CONVL_NC(false, false, true);
        else SG_CONVL_NC(false, false, false);
    } else if (ks == 3) {
        if (out_f32) SG_CONV_NC(3, false, true, false);
        else if (relu) SG_CONV_NC(3, true, false, false);
        else if (mask) SG_CONV_NC(3, false, false, true);
        else SG_CONV_NC(3, false, false, false);
    } else if (ks == 1) {
        if (out_f32) SG_CONV_NC(1, false, true, false);
        else if (relu) SG_CONV_NC(1, true, false, false);
        else if (mask) SG_CONV_NC(1, false, false, true);
        else SG_CONV_NC(1, false, false, false);
    } else {
        return fail(SG_EINVAL, "net: kernel size must be 1 or 3");
    }
#undef SG_CONVL_NC
#undef SG_CONVL
#undef SG_CONV_NC
#undef SG_CONV
    SG_HIP(hipGetLastError());
    return SG_OK;
}

long long net_wgrad_scratch(int Cout, int Cin, int ks, int H, int Wd, int batch) {
    const int nchunk = (H * Wd + WG_CHUNK - 1) / WG_CHUNK;
    return (long long)batch * nchunk * Cout * ks * ks * Cin;
}

int net_wgrad(const uint16_t* dZ, int Cout, const uint16_t* X, int Cin, int H, int Wd, int batch, int ks, int co_real,
              int ci_real, float* scratch, float* gW, float* gb, float* scratch_b, hipStream_t st) {
    const int nchunk = (H * Wd + WG_CHUNK - 1) / WG_CHUNK;
    const int KK = ks * ks;
    const dim3 grid((unsigned)(Cin / 32 * KK), (unsigned)(Cout / 32), (unsigned)(batch * nchunk)), blk(256);
    {
        KScope k(SG_K_NET, 2.0 * H * Wd * (double)batch * Cout * Cin * KK, st);
        if (ks == 3) hipLaunchKernelGGL(k_wgrad<3>, grid, blk, 0, st, dZ, Cout, X, Cin, H, Wd, nchunk, scratch);
        else hipLaunchKernelGGL(k_wgrad<1>, grid, blk, 0, st, dZ, Cout, X, Cin, H, Wd, nchunk, scratch);
        SG_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(grid_of((long long)co_real * KK * ci_real)), dim3(256), 0, st, scratch,
                       batch * nchunk, Cout, KK, Cin, co_real, ci_real, gW);
    SG_HIP(hipGetLastError());
    const long long npix = (long long)batch * H * Wd;
    const int per = COLSUM_PER;
    const int nb = (int)((npix + per - 1) / per);
    if (Cout > 256 || Cout % 8) return fail(SG_EINVAL, "net: channel count unsuitable for the bias reduction");
    hipLaunchKernelGGL(k_colsum, dim3(nb), dim3(256), 0, st, dZ, npix, Cout, per, scratch_b);
    hipLaunchKernelGGL(k_colsum_reduce, dim3(co_real), dim3(256), 0, st, scratch_b, nb, Cout, co_real, gb);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

long long net_colsum_scratch(int Cout, int H, int Wd, int batch) {
    return ((long long)batch * H * Wd + COLSUM_PER - 1) / COLSUM_PER * Cout;
}

int net_pool(const uint16_t* in, uint16_t* out, int Hl, int Wl, int C, int batch, hipStream_t st) {
    const long long n = (long long)batch * Hl * Wl * C;
    hipLaunchKernelGGL(k_pool, dim3(grid_of(n)), dim3(256), 0, st, in, out, Hl, Wl, C, n);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int net_up_concat(const uint16_t* U, int Cu, const uint16_t* S, int Cs, uint16_t* out, int H, int Wd, int batch,
                  hipStream_t st) {
    const long long n = (long long)batch * H * Wd * (Cu + Cs);
    hipLaunchKernelGGL(k_up_concat, dim3(grid_of(n)), dim3(256), 0, st, U, Cu, S, Cs, out, H, Wd, n);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int net_up_bwd(const uint16_t* dC, int C, int Cu, const uint16_t* mask, uint16_t* out, int Hl, int Wl, int batch,
               hipStream_t st) {
    const long long n = (long long)batch * Hl * Wl * Cu;
    hipLaunchKernelGGL(k_up_bwd, dim3(grid_of(n)), dim3(256), 0, st, dC, C, Cu, mask, out, Hl, Wl, n);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int net_skip_bwd(const uint16_t* dC, int Ccat, int Cu, const uint16_t* dP, const uint16_t* mask, uint16_t* out, int H,
                 int Wd, int C, int batch, hipStream_t st) {
    const long long n = (long long)batch * H * Wd * C;
    hipLaunchKernelGGL(k_skip_bwd, dim3(grid_of(n)), dim3(256), 0, st, dC, Ccat, Cu, dP, mask, out, H, Wd, C, n);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int net_pack(const double2* r, const double2* rnorm, int Q, int n, int H, const double* kf, int s, double kbar, int Cp,
             uint16_t* out, hipStream_t st) {
    hipLaunchKernelGGL(k_pack, dim3(grid_of((long long)H * H * Cp)), dim3(256), 0, st, r, rnorm, Q, n, H, kf, s, kbar, Cp,
                       out);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int net_unpack_add(const float* y, int Cp, const double2* znorm, int Q, int n, int H, double2* z, hipStream_t st) {
    hipLaunchKernelGGL(k_unpack_add, dim3(grid_of((long long)Q * n * n)), dim3(256), 0, st, y, Cp, znorm, Q, n, H, z);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int net_pack_target(const double2* c, const double2* znorm, int Q, int n, int H, int Cp, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_pack_target, dim3(grid_of((long long)H * H * Cp)), dim3(256), 0, st, c, znorm, Q, n, H, Cp, out);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int net_to_bf16(const float* in, int C, uint16_t* out, int Cp, long long npix, hipStream_t st) {
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_of(npix * Cp)), dim3(256), 0, st, in, C, out, Cp, npix);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int net_pad_f32(const float* in, int C, float* out, int Cp, long long npix, hipStream_t st) {
    hipLaunchKernelGGL(k_pad_f32, dim3(grid_of(npix * Cp)), dim3(256), 0, st, in, C, out, Cp, npix);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int net_unpad_f32(const float* in, int Cp, float* out, int C, long long npix, hipStream_t st) {
    hipLaunchKernelGGL(k_unpad_f32, dim3(grid_of(npix * C)), dim3(256), 0, st, in, Cp, out, C, npix);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int net_mse(const float* y, const float* t, long long npix, int Cp, int C, double inv_count, uint16_t* dy, float* partial,
            int nblocks, hipStream_t st) {
    hipLaunchKernelGGL(k_mse, dim3(nblocks), dim3(256), 0, st, y, t, npix, Cp, C, inv_count, dy, partial);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int net_adam(float* th, float* m, float* v, const float* g, long long n, float lr, float b1, float b2, float eps, int t,
             hipStream_t st) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(grid_of(n)), dim3(256), 0, st, th, m, v, g, n, lr, b1, b2, eps, c1, c2);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int net_weights(const float* th, int co_real, int ci_real, int ks, int Coutp, int Cinp, uint16_t* wf, uint16_t* wb,
                float* bias, hipStream_t st) {
    const long long n = (long long)Coutp * ks * ks * Cinp;
    hipLaunchKernelGGL(k_weights, dim3(grid_of(n)), dim3(256), 0, st, th, co_real, ci_real, ks * ks, Coutp, Cinp, wf, wb,
                       bias);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

}  // namespace sgi
