// Block solves with a spatially varying mean wavenumber (Section 7, eqs.
// stochastic_wavenumber_k123 / wavenumber_k123): the mean block S(ξ̄) = S(k_0) of the
// preconditioners A_0 and M_0 (Section 5, eq. bar_A; eq. M) is then no longer separable,
// so the fast diagonalisation of the constant-k̄ case does not apply.  Instead the block
// is factorised exactly, as the paper factorises it (an LU of one diagonal block, reused
// for all Q blocks, Section 6.3), in the form that suits the GPU: block Gaussian
// elimination over the grid lines.
//
// With the nodes ordered x fastest (Theorem A.3 ordering), the 2D block of Theorem A.4 is
// block tridiagonal over the lines y_j (j = 0..n-1), each line a block of L = n unknowns:
//     A_j = d_j T + T_jj D - i diag(e k_0 / h) - c diag(w k_0²)      (on line j)
//     B   = T_{j,j±1} D = -(1/h²) D                                    (lines j, j±1)
// with T the 1D absorbing Laplacian, D = diag(d), d = (½,1,...,1,½), and c = 1 (A_0) or
// 1+iβ (M_0, shift on the k² term only).  In 1D the same recursion runs over single
// nodes (L = 1, B = -1/h²).  Block LU without pivoting between lines:
//     Ŝ_0 = A_0,   Ŝ_j = A_j - B Ŝ_{j-1}^{-1} B,   E_j = Ŝ_j^{-1} (dense L×L, pivoted LU on the host)
//     forward   y_0 = E_0 r_0,   y_j = E_j (r_j - B y_{j-1})
//     backward  x_{n-1} = y_{n-1},   x_j = y_j - E_j B x_{j+1}.
// The factors are checked at setup by solving a random system and measuring the residual
// with the sparse block itself.  Each line step is a dense L×L matrix-vector product per
// right-hand side, and a step has to wait for the previous one, so the sweep is a chain of
// 2n-1 dependent steps whose length is set by how fast one CU can stream E_j (L·L·16 bytes)
// from L2 or the Infinity Cache.
//   k_line_pipe (L <= 132): one workgroup per right-hand side; the rows of E_j are spread
//     over the waves (16 per wave) and the k range of a row over the four 16-lane groups of
//     a wave, whose partial sums are joined by lane exchanges (no LDS, one barrier per
//     step).  Each lane keeps its KCM entries of the matrix in registers and loads those of
//     the next step's matrix as it consumes the current ones, so the loads of step s+1 are in
//     flight during the reduction and barrier of step s.  The k groups cover 4·KCM >= L rows;
//     the rows past L-1 (the next matrix, or zero padding after the last one) meet t = 0.
//   k_line_lu (longer lines): NC right-hand sides per workgroup, the k range split over KS
//     thread groups joined through LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <functional>
#include <random>
#include <thread>
#include <vector>

#include "sg_internal.h"

namespace sgi {

namespace {

constexpr int LT = 512;   // threads per workgroup (lines of up to 512 nodes)
constexpr int NC = 2;     // right-hand sides (PC blocks) per workgroup

// E: [nl][L][L] with E[j][k][i] = (E_j)_{ik} (column k of E_j contiguous over i);
// b: [L] the diagonal of B; X: [Q][nl][L] complex, in: r (may alias X).
__global__ __launch_bounds__(LT) void k_line_lu(const double2* __restrict__ E, const double* __restrict__ b,
                                                const double2* r, double2* X, int L, int nl, int Q, int KS,
                                                long long P) {
    __shared__ double2 t[NC][LT];
    __shared__ double2 part[8][NC][LT / 2];   // partial sums of the k groups 1..KS-1 (KS·L <= 1024 rows)
    const int tid = threadIdx.x;
    const int KC = (L + KS - 1) / KS;
    const int ks = tid / L, i = tid - ks * L;
    const bool row = ks < KS;                 // thread (ks, i) owns row i of k group ks
    const bool lead = ks == 0;                // ... and group 0 owns the row's result
    const int k0 = ks * KC, k1 = min(L, k0 + KC);
    const int q0 = blockIdx.x * NC;
    const double bi = lead ? b[i] : 0.0;
    double2 keep[NC];                         // y_{j-1} (forward) / x_{j+1} (backward) of row i
#pragma unroll
    for (int c = 0; c < NC; ++c) keep[c] = make_double2(0.0, 0.0);

    // acc[c] = Σ_{k in this group} E_j[i][k] t[c][k]; group 0 adds the other groups' parts
    auto matvec = [&](int j, double2 (&acc)[NC]) {
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = make_double2(0.0, 0.0);
        if (row) {
            const double2* Ej = E + (long long)j * L * L + i;
#pragma unroll 4
            for (int k = k0; k < k1; ++k) {
                const double2 e = Ej[(long long)k * L];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const double2 tv = t[c][k];
                    acc[c].x = fma(e.x, tv.x, fma(-e.y, tv.y, acc[c].x));
                    acc[c].y = fma(e.x, tv.y, fma(e.y, tv.x, acc[c].y));
                }
            }
            if (!lead)
#pragma unroll
                for (int c = 0; c < NC; ++c) part[ks - 1][c][i] = acc[c];
        }
        __syncthreads();
        if (lead && row)
            for (int g = 1; g < KS; ++g)
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    acc[c].x += part[g - 1][c][i].x;
                    acc[c].y += part[g - 1][c][i].y;
                }
    };

    for (int j = 0; j < nl; ++j) {
        if (lead && row)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int q = q0 + c;
                double2 v = make_double2(0.0, 0.0);
                if (q < Q) v = r[(long long)q * P + (long long)j * L + i];
                t[c][i] = make_double2(fma(-bi, keep[c].x, v.x), fma(-bi, keep[c].y, v.y));
            }
        __syncthreads();
        double2 acc[NC];
        matvec(j, acc);
        if (lead && row)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                keep[c] = acc[c];
                if (q0 + c < Q) X[(long long)(q0 + c) * P + (long long)j * L + i] = acc[c];
            }
        __syncthreads();   // t and part are rewritten by the next step
    }
    for (int j = nl - 2; j >= 0; --j) {
        if (lead && row)
#pragma unroll
            for (int c = 0; c < NC; ++c) t[c][i] = make_double2(bi * keep[c].x, bi * keep[c].y);
        __syncthreads();
        double2 acc[NC];
        matvec(j, acc);
        if (lead && row)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (q0 + c < Q) {
                    double2* xp = X + (long long)(q0 + c) * P + (long long)j * L + i;
                    const double2 y = *xp;   // y_j, written by this thread in the forward sweep
                    keep[c] = make_double2(y.x - acc[c].x, y.y - acc[c].y);
                    *xp = keep[c];
                }
            }
        __syncthreads();
    }
}

constexpr int PIPE_LMAX = 132;   // longest line of the pipelined kernel (4 groups of 33 rows)

// Row-block base, advanced by one row and hidden from the optimiser: the bases are formed one
// after another next to their loads (formed all at once they would hold one register pair
// per row for the whole step).
__device__ __forceinline__ const double2* next_row(const double2* p, int L) {
    p += L;
    asm volatile("" : "+s"(p));
    return p;
}
// A wave-uniform base plus a 32-bit per-lane byte offset (one offset register for all loads).
__device__ __forceinline__ double2 ld_off(const double2* base, unsigned boff) {
    return *reinterpret_cast<const double2*>(reinterpret_cast<const char*>(base) + boff);
}

template <int KCM>
__global__ __launch_bounds__(576) void k_line_pipe(const double2* __restrict__ E, const double* __restrict__ b,
                                                   const double2* r, double2* X, int L, int nl, long long P) {
    constexpr int KG = 4, RW = 64 / KG;
    __shared__ double2 t[2][PIPE_LMAX];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane / RW, ii = lane - g * RW;
    const int i = w * RW + ii;
    const bool rowok = i < L;
    const int ic = rowok ? i : L - 1;
    const bool lead = g == 0 && rowok;        // lane (0, i) owns row i's result
    const int k0 = g * KCM;                   // this lane's rows k0 .. k0+KCM-1 of E_j
    const long long q = blockIdx.x;
    const double bi = b[ic];
    const double2* rq = r + q * P + ic;
    double2* xq = X + q * P + ic;
    const int nsteps = 2 * nl - 1;            // forward j = 0..nl-1, then backward j = nl-2..0
    auto mat = [&](int s) { return s < nl ? s : 2 * nl - 2 - s; };
    const unsigned voff = (unsigned)(k0 * L + ic) * 16u;
    double2 e[KCM];
    {
        const double2* Ep = E;
#pragma unroll
        for (int m = 0; m < KCM; ++m) {
            e[m] = ld_off(Ep, voff);
            Ep = next_row(Ep, L);
        }
    }
    for (int k = L + (int)threadIdx.x; k < KG * KCM; k += blockDim.x) t[0][k] = t[1][k] = make_double2(0.0, 0.0);
    if (lead) t[0][i] = rq[0];
    // nxt: the right-hand side of the next forward step, then y_j of the next backward step
    double2 nxt = lead && nl > 1 ? rq[(long long)L] : make_double2(0.0, 0.0);
    __syncthreads();
    int buf = 0;
    for (int s = 0; s < nsteps; ++s) {
        const bool fwd = s < nl;
        const int j = mat(s);
        const double2 cur = nxt;
        if (lead) {
            if (fwd && j + 2 < nl) nxt = rq[(long long)(j + 2) * L];
            else if (fwd && j == nl - 1 && nl >= 2) nxt = xq[(long long)(nl - 2) * L];
            else if (!fwd && j >= 1) nxt = xq[(long long)(j - 1) * L];
        }
        double2 acc = make_double2(0.0, 0.0);
        // the next step's matrix (the last step reloads its own: no branch in the loop)
        const double2* Ep = E + (long long)mat(s + 1 < nsteps ? s + 1 : s) * L * L;
#pragma unroll
        for (int m = 0; m < KCM; ++m) {
            const double2 tv = t[buf][k0 + m];
            acc.x = fma(e[m].x, tv.x, fma(-e[m].y, tv.y, acc.x));
            acc.y = fma(e[m].x, tv.y, fma(e[m].y, tv.x, acc.y));
            e[m] = ld_off(Ep, voff);
            Ep = next_row(Ep, L);
        }
#pragma unroll
        for (int off = RW; off < 64; off <<= 1) {
            acc.x += __shfl_xor(acc.x, off, 64);
            acc.y += __shfl_xor(acc.y, off, 64);
        }
        if (lead) {
            double2 x;
            if (fwd) {   // y_j = E_j (r_j - B y_{j-1}); then r_{j+1} - B y_j, or B y_{n-1} to start backward
                x = acc;
                t[buf ^ 1][i] = j + 1 < nl ? make_double2(fma(-bi, x.x, cur.x), fma(-bi, x.y, cur.y))
                                           : make_double2(bi * x.x, bi * x.y);
            } else {     // x_j = y_j - E_j B x_{j+1}; then B x_j
                x = make_double2(cur.x - acc.x, cur.y - acc.y);
                t[buf ^ 1][i] = make_double2(bi * x.x, bi * x.y);
            }
            xq[(long long)j * L] = x;
        }
        buf ^= 1;
        __syncthreads();
    }
}

// Rows of each line factor the pipelined kernel reads (4·KCM >= L), or 0 for the LDS kernel.
int pipe_kcm(int L) {
    if (L <= 32) return 8;
    if (L <= 64) return 16;
    if (L <= PIPE_LMAX) return 33;
    return 0;
}

// ---- host factorisation -----------------------------------------------------------

void parallel_for(int n, int nthreads, const std::function<void(int, int)>& fn) {
    nthreads = std::max(1, std::min(nthreads, n));
    if (nthreads == 1) {
        fn(0, n);
        return;
    }
    std::vector<std::thread> th;
    const int chunk = (n + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        const int a = t * chunk, e = std::min(n, a + chunk);
        if (a < e) th.emplace_back(fn, a, e);
    }
    for (auto& x : th) x.join();
}

// In-place inverse of the L×L row-major matrix M (LU with partial pivoting, then the L
// unit right-hand sides); false if a pivot is zero.
bool invert(int L, std::vector<cplx>& M, std::vector<cplx>& inv, int nthreads) {
    std::vector<int> perm(L);
    for (int i = 0; i < L; ++i) perm[i] = i;
    for (int k = 0; k < L; ++k) {
        int p = k;
        double best = std::abs(M[(size_t)k * L + k]);
        for (int i = k + 1; i < L; ++i) {
            const double v = std::abs(M[(size_t)i * L + k]);
            if (v > best) { best = v; p = i; }
        }
        if (best == 0.0) return false;
        if (p != k) {
            std::swap_ranges(M.begin() + (size_t)k * L, M.begin() + (size_t)(k + 1) * L, M.begin() + (size_t)p * L);
            std::swap(perm[k], perm[p]);
        }
        const cplx piv = M[(size_t)k * L + k];
        const cplx* rk = &M[(size_t)k * L];
        auto upd = [&](int a, int e) {
            for (int i = k + 1 + a; i < k + 1 + e; ++i) {
                cplx* ri = &M[(size_t)i * L];
                const cplx l = ri[k] / piv;
                ri[k] = l;
                for (int c = k + 1; c < L; ++c) ri[c] -= l * rk[c];
            }
        };
        const int rows = L - k - 1;
        if (rows * (L - k) > 16384) parallel_for(rows, nthreads, upd);
        else upd(0, rows);
    }
    inv.assign((size_t)L * L, 0.0);
    // column c of the inverse solves L U x = P e_c
    parallel_for(L, nthreads, [&](int a, int e) {
        std::vector<cplx> x(L);
        for (int c = a; c < e; ++c) {
            for (int i = 0; i < L; ++i) x[i] = perm[i] == c ? 1.0 : 0.0;
            for (int i = 0; i < L; ++i) {
                cplx s = x[i];
                const cplx* ri = &M[(size_t)i * L];
                for (int k = 0; k < i; ++k) s -= ri[k] * x[k];
                x[i] = s;
            }
            for (int i = L - 1; i >= 0; --i) {
                cplx s = x[i];
                const cplx* ri = &M[(size_t)i * L];
                for (int k = i + 1; k < L; ++k) s -= ri[k] * x[k];
                x[i] = s / ri[i];
            }
            for (int i = 0; i < L; ++i) inv[(size_t)i * L + c] = x[i];
        }
    });
    return true;
}

}  // namespace

// Diagonal-block entries of S(k_0) on line j (see the header comment): the tridiagonal
// A_j as (lower, diagonal, upper) and the line coupling b.
static void line_block(const Ctx* c, const std::vector<double>& k0, cplx shift, int j, std::vector<cplx>& lo,
                       std::vector<cplx>& di, std::vector<cplx>& up) {
    const int n = c->n, L = c->line_L;
    const double ih2 = 1.0 / (c->h * c->h);
    auto dw = [&](int i) { return (i == 0 || i == n - 1) ? 0.5 : 1.0; };
    auto tdiag = [&](int i) { return (i == 0 || i == n - 1) ? ih2 : 2.0 * ih2; };
    lo.assign(L, 0.0);
    di.assign(L, 0.0);
    up.assign(L, 0.0);
    for (int i = 0; i < L; ++i) {
        const long long p = (long long)j * L + i;
        double w, e, lap;
        if (c->dim == 2) {
            w = dw(i) * dw(j);
            e = (i == 0 || j == 0 || i == n - 1 || j == n - 1) ? 1.0 : 0.0;
            lap = dw(j) * tdiag(i) + tdiag(j) * dw(i);
            if (i > 0) lo[i] = -dw(j) * ih2;
            if (i < L - 1) up[i] = -dw(j) * ih2;
        } else {
            w = dw(j);
            e = (j == 0 || j == n - 1) ? 1.0 : 0.0;
            lap = tdiag(j);
        }
        di[i] = lap - cplx(0.0, e * k0[p] / c->h) - shift * (w * k0[p] * k0[p]);
    }
}

int build_line_factors(Ctx* c, const double* k0_host) {
    const int n = c->n;
    const int L = c->dim == 2 ? n : 1;
    const int nl = n;
    c->line_L = L;
    c->line_nl = nl;
    const double ih2 = 1.0 / (c->h * c->h);
    std::vector<double> k0(k0_host, k0_host + c->P);
    std::vector<double> bl(L);
    for (int i = 0; i < L; ++i) bl[i] = c->dim == 2 ? -((i == 0 || i == n - 1) ? 0.5 : 1.0) * ih2 : -ih2;
    const int nthreads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    for (int t = 0; t < 2; ++t) {
        const cplx shift = t == 0 ? cplx(1.0, 0.0) : cplx(1.0, c->beta);
        std::vector<cplx> Einv((size_t)nl * L * L);   // row-major inverses, [j][i][k]
        std::vector<cplx> M((size_t)L * L), inv, lo, di, up;
        for (int j = 0; j < nl; ++j) {
            line_block(c, k0, shift, j, lo, di, up);
            std::fill(M.begin(), M.end(), cplx(0.0));
            for (int i = 0; i < L; ++i) {
                M[(size_t)i * L + i] = di[i];
                if (i > 0) M[(size_t)i * L + i - 1] = lo[i];
                if (i < L - 1) M[(size_t)i * L + i + 1] = up[i];
            }
            if (j > 0) {
                const cplx* Ep = &Einv[(size_t)(j - 1) * L * L];
                for (int i = 0; i < L; ++i)
                    for (int k = 0; k < L; ++k) M[(size_t)i * L + k] -= bl[i] * Ep[(size_t)i * L + k] * bl[k];
            }
            if (!invert(L, M, inv, nthreads)) return fail(SG_ESETUP, "singular line block in the varying-mean factorisation");
            std::copy(inv.begin(), inv.end(), Einv.begin() + (size_t)j * L * L);
        }
        // validation: solve S x = r for a random r on the host and measure ||S x - r|| / ||r||
        std::mt19937_64 rng(12345 + t);
        std::normal_distribution<double> nd;
        const long long P = c->P;
        std::vector<cplx> rv(P), x(P), tv(L);
        for (auto& v : rv) v = cplx(nd(rng), nd(rng));
        for (int j = 0; j < nl; ++j) {
            for (int i = 0; i < L; ++i) tv[i] = rv[(size_t)j * L + i] - (j > 0 ? bl[i] * x[(size_t)(j - 1) * L + i] : 0.0);
            const cplx* Ej = &Einv[(size_t)j * L * L];
            for (int i = 0; i < L; ++i) {
                cplx s = 0;
                for (int k = 0; k < L; ++k) s += Ej[(size_t)i * L + k] * tv[k];
                x[(size_t)j * L + i] = s;
            }
        }
        for (int j = nl - 2; j >= 0; --j) {
            for (int k = 0; k < L; ++k) tv[k] = bl[k] * x[(size_t)(j + 1) * L + k];
            const cplx* Ej = &Einv[(size_t)j * L * L];
            for (int i = 0; i < L; ++i) {
                cplx s = 0;
                for (int k = 0; k < L; ++k) s += Ej[(size_t)i * L + k] * tv[k];
                x[(size_t)j * L + i] -= s;
            }
        }
        double rn = 0, en = 0;
        for (int j = 0; j < nl; ++j) {
            line_block(c, k0, shift, j, lo, di, up);
            for (int i = 0; i < L; ++i) {
                const size_t p = (size_t)j * L + i;
                cplx s = di[i] * x[p];
                if (i > 0) s += lo[i] * x[p - 1];
                if (i < L - 1) s += up[i] * x[p + 1];
                if (j > 0) s += bl[i] * x[p - L];
                if (j < nl - 1) s += bl[i] * x[p + L];
                en += std::norm(s - rv[p]);
                rn += std::norm(rv[p]);
            }
        }
        const double rel = std::sqrt(en / rn);
        c->line_check[t] = rel;
        if (!(rel < 1e-8)) {
            char msg[160];
            std::snprintf(msg, sizeof msg, "varying-mean line factorisation failed its check: residual %.3e", rel);
            return fail(SG_ESETUP, msg);
        }
        // device layout E[j][k][i]
        std::vector<double2> dev((size_t)nl * L * L);
        for (int j = 0; j < nl; ++j)
            for (int i = 0; i < L; ++i)
                for (int k = 0; k < L; ++k) {
                    const cplx v = Einv[((size_t)j * L + i) * L + k];
                    dev[((size_t)j * L + k) * L + i] = make_double2(v.real(), v.imag());
                }
        // zero padding after the last factor: the pipelined kernel's last k group reads up to
        // 4·KCM - L rows past the end of a factor
        const int kcm = pipe_kcm(L);
        const size_t pad = kcm ? (size_t)std::max(0, 4 * kcm - L) * L : 0;
        SG_HIP(setup_alloc(&c->d_lineE[t], (dev.size() + pad) * sizeof(double2)));
        if (int rc_ = upload(c->d_lineE[t], dev.data(), dev.size() * sizeof(double2))) return rc_;
        if (pad)
            if (int rc_ = upload_zero(c->d_lineE[t] + dev.size(), pad * sizeof(double2))) return rc_;
    }
    SG_HIP(setup_alloc(&c->d_lineb, (size_t)L * sizeof(double)));
    if (int rc_ = upload(c->d_lineb, bl.data(), (size_t)L * sizeof(double))) return rc_;
    return SG_OK;
}

int launch_line(Ctx* c, int pc, const double2* r, double2* z, hipStream_t st) {
    const int L = c->line_L, nl = c->line_nl;
    if (L < 1 || L > LT) return fail(SG_EINVAL, "varying-mean block solve: line length out of range");
    const double2* E = c->d_lineE[pc == SG_PC_MEAN ? 0 : 1];
    const int kcm = pipe_kcm(L);
    if (kcm) {
        // every workgroup streams all 2n-1 factors once (from L2 / the Infinity Cache)
        KScope ks(SG_K_TRI, 16.0 * (2.0 * nl - 1.0) * L * L * c->Q + 48.0 * (double)c->nvec, st);
        const dim3 grid((unsigned)c->Q), block((unsigned)(64 * ((L + 15) / 16)));
        if (kcm == 8) hipLaunchKernelGGL(k_line_pipe<8>, grid, block, 0, st, E, c->d_lineb, r, z, L, nl, c->P);
        else if (kcm == 16) hipLaunchKernelGGL(k_line_pipe<16>, grid, block, 0, st, E, c->d_lineb, r, z, L, nl, c->P);
        else hipLaunchKernelGGL(k_line_pipe<33>, grid, block, 0, st, E, c->d_lineb, r, z, L, nl, c->P);
        SG_HIP(hipGetLastError());
        return SG_OK;
    }
    const int KS = std::max(1, std::min(8, LT / L));   // KS > 1 only for L <= 256: the partial sums fit
    const int nblk = (c->Q + NC - 1) / NC;
    KScope ks(SG_K_TRI, 2.0 * 16.0 * (double)nl * L * L * nblk + 48.0 * (double)c->nvec, st);
    hipLaunchKernelGGL(k_line_lu, dim3(nblk), dim3(LT), 0, st, E, c->d_lineb, r, z, L, nl, c->Q, KS, c->P);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

}  // namespace sgi
