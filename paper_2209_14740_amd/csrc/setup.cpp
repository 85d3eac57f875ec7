// Host-side setup of the SG Helmholtz operator (FP64, validated), then upload.
//
//  * Chaos basis: multi-indices of total degree <= r in s variables, graded and
//    descending-lexicographic within a degree (Section 2.3).
//  * Galerkin coupling: with k = k_0 + Σ k_ℓ ξ_ℓ (eq. random_wavenumber) and
//    ξ = φ_1/√3, ξ² = 1/3 + 2φ_2/(3√5) for the orthonormal Legendre φ_n, the
//    products k and k² are finite sums Σ_γ κ_γ(x) Ψ_γ(ξ) over the multi-indices γ
//    of degree <= 1 and <= 2.  Hence (eqs. b_ij, c_ij)
//        b_ij(x) = Σ_γ κ1_γ(x) E[Ψ_γ φ_i φ_j],   c_ij(x) = Σ_γ κ2_γ(x) E[Ψ_γ φ_i φ_j],
//    and E[Ψ_γ φ_i φ_j] = Π_ℓ t(γ_ℓ, α_iℓ, α_jℓ) with the univariate triple product
//    t(c,a,b) = E[φ_c φ_a φ_b] = sqrt((2a+1)(2b+1)(2c+1)) · (a b c; 0 0 0)², the squared
//    Wigner 3j symbol (Adams-Neumann linearisation of Legendre products).  Exact zeros
//    come from its parity and triangle rules.
//  * Fields: D2_γ = w·κ2_γ (k² term with the boundary weights of Theorem A.4) and
//    D1_γ = (e/h)·κ1_γ (absorbing-boundary term, Theorem A.2 / A.4).
//  * Mean block: with k_0 = k̄ constant, S(ξ̄) = D⊗S_1 + S_1⊗D in 2D, where
//    S_1 = T - i(k̄/h)E_1 - (c/2)D, E_1 = diag(1,0,...,0,1), c = k̄² (A_0) or (1+iβ)k̄²
//    (M_0, eq. M); in 1D S(ξ̄) = T - i(k̄/h)E_1 - cD (Theorem A.2, Remark 6.1).
//    The generalised eigenpairs (T - i(k̄/h)E_1) v_a = μ_a D v_a, normalised v_aᵀ D v_a = 1
//    (complex symmetric, unconjugated), do not depend on c.  Writing the block vector
//    as X[x,y], S(ξ̄)X = S_1 X D + D X S_1; substituting X = Ṽ W gives for every a the
//    tridiagonal system along y (T - i(k̄/h)E_1 + (μ_a - c) D) w_a = (Ṽᵀ R)_a.  The
//    preconditioner is thus one dense transform along x, Na pivoted tridiagonal solves
//    along y, and the inverse transform (fast diagonalisation in one direction,
//    after Lynch, Rice & Thomas 1964).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>

#include "sg_internal.h"

namespace sgi {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}
const char* last_error() { return g_last_error.c_str(); }

// ---------------------------------------------------------------- basis

static void enum_level(int s, int d, std::vector<int>& cur, std::vector<int>& out) {
    // all tuples of length s with sum d, first component descending
    int pos = (int)cur.size();
    if (pos == s - 1) {
        cur.push_back(d);
        out.insert(out.end(), cur.begin(), cur.end());
        cur.pop_back();
        return;
    }
    for (int a = d; a >= 0; --a) {
        cur.push_back(a);
        enum_level(s, d - a, cur, out);
        cur.pop_back();
    }
}

static std::vector<int> make_basis(int s, int r) {
    std::vector<int> out, cur;
    for (int d = 0; d <= r; ++d) enum_level(s, d, cur, out);
    return out;
}

static long double lfactorial(int n) {
    long double f = 1.0L;
    for (int i = 2; i <= n; ++i) f *= (long double)i;
    return f;
}

// t(c,a,b) = E[φ_c φ_a φ_b] for orthonormal Legendre φ and ξ ~ U[-1,1].
static double triple(int c, int a, int b) {
    int tot = a + b + c;
    if (tot & 1) return 0.0;
    int g = tot / 2;
    if (a > g || b > g || c > g) return 0.0;
    long double w3 = lfactorial(2 * g - 2 * a) * lfactorial(2 * g - 2 * b) * lfactorial(2 * g - 2 * c) /
                     lfactorial(2 * g + 1);
    long double ratio = lfactorial(g) / (lfactorial(g - a) * lfactorial(g - b) * lfactorial(g - c));
    w3 *= ratio * ratio;
    return (double)(sqrtl((long double)(2 * a + 1) * (2 * b + 1) * (2 * c + 1)) * w3);
}

static void build_coupling(const std::vector<int>& alpha, int Q, int s,
                           const std::vector<std::vector<int>>& gammas, Coupling& cp) {
    cp.nfield = (int)gammas.size();
    cp.pair_ptr.assign(1, 0);
    cp.pair_j.clear();
    cp.term_ptr.assign(1, 0);
    cp.term_field.clear();
    cp.term_val.clear();
    for (int i = 0; i < Q; ++i) {
        for (int j = 0; j < Q; ++j) {
            int nterm = 0;
            for (int g = 0; g < (int)gammas.size(); ++g) {
                double v = 1.0;
                for (int l = 0; l < s && v != 0.0; ++l)
                    v *= triple(gammas[g][l], alpha[i * s + l], alpha[j * s + l]);
                if (v != 0.0) {
                    cp.term_field.push_back(g);
                    cp.term_val.push_back(v);
                    ++nterm;
                }
            }
            if (nterm) {
                cp.pair_j.push_back(j);
                cp.term_ptr.push_back((int)cp.term_field.size());
            }
        }
        cp.pair_ptr.push_back((int)cp.pair_j.size());
    }
}

// ------------------------------------------------- complex symmetric eigen

// Eigenvalues of the complex symmetric tridiagonal matrix (diag d, off-diagonal e with
// e[i] coupling rows i and i+1) by the implicit QL iteration with complex orthogonal
// plane rotations (Bowdler-Martin-Reinsch-Wilkinson 1968 QL in the complex symmetric
// form of Cullum & Willoughby).  Returns false if an eigenvalue fails to converge.
static bool ql_eigenvalues(std::vector<cplx>& d, std::vector<cplx> e) {
    const int n = (int)d.size();
    e.resize(n);
    e[n - 1] = 0.0;
    const double eps = 2.2e-16;
    for (int l = 0; l < n; ++l) {
        int iter = 0, m;
        do {
            for (m = l; m < n - 1; ++m) {
                double dd = std::abs(d[m]) + std::abs(d[m + 1]);
                if (std::abs(e[m]) <= eps * dd) break;
            }
            if (m != l) {
                if (++iter > 200) return false;
                cplx g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                cplx r = std::sqrt(g * g + 1.0);
                cplx gp = g + r, gm = g - r;
                g = d[m] - d[l] + e[l] / (std::abs(gp) >= std::abs(gm) ? gp : gm);
                cplx s = 1.0, c = 1.0, p = 0.0;
                int i;
                bool early = false;
                for (i = m - 1; i >= l; --i) {
                    cplx f = s * e[i], b = c * e[i];
                    r = std::sqrt(f * f + g * g);
                    e[i + 1] = r;
                    if (std::abs(r) == 0.0) {
                        d[i + 1] -= p;
                        e[m] = 0.0;
                        early = true;
                        break;
                    }
                    s = f / r;
                    c = g / r;
                    g = d[i + 1] - p;
                    r = (d[i] - g) * s + 2.0 * c * b;
                    p = s * r;
                    d[i + 1] = g + p;
                    g = c * r - b;
                }
                if (early) continue;
                d[l] -= p;
                e[l] = g;
                e[m] = 0.0;
            }
        } while (m != l);
    }
    return true;
}

// Pivoted LU of a complex tridiagonal matrix (sub dl, diag d, super du), row-partial
// pivoting.  On exit: dl = multipliers, d = U diagonal, du = U first super-diagonal,
// du2 = U second super-diagonal, piv[i] = 1 when rows i, i+1 were exchanged.
static bool tri_lu(int n, std::vector<cplx>& dl, std::vector<cplx>& d, std::vector<cplx>& du,
                   std::vector<cplx>& du2, std::vector<uint8_t>& piv) {
    du2.assign(std::max(n - 2, 0), 0.0);
    piv.assign(std::max(n - 1, 0), 0);
    for (int i = 0; i < n - 1; ++i) {
        if (std::abs(d[i]) >= std::abs(dl[i])) {
            if (d[i] == 0.0) return false;
            cplx l = dl[i] / d[i];
            dl[i] = l;
            d[i + 1] -= l * du[i];
        } else {
            cplx l = d[i] / dl[i];
            piv[i] = 1;
            d[i] = dl[i];
            dl[i] = l;
            cplx old_d1 = d[i + 1];
            cplx old_u = du[i];
            du[i] = old_d1;
            d[i + 1] = old_u - l * old_d1;
            if (i < n - 2) {
                du2[i] = du[i + 1];
                du[i + 1] = -l * du[i + 1];
            }
        }
    }
    return d[n - 1] != 0.0;
}

static void tri_solve(int n, const std::vector<cplx>& dl, const std::vector<cplx>& d,
                      const std::vector<cplx>& du, const std::vector<cplx>& du2,
                      const std::vector<uint8_t>& piv, std::vector<cplx>& b) {
    for (int i = 0; i < n - 1; ++i) {
        if (piv[i]) std::swap(b[i], b[i + 1]);
        b[i + 1] -= dl[i] * b[i];
    }
    b[n - 1] /= d[n - 1];
    if (n >= 2) b[n - 2] = (b[n - 2] - du[n - 2] * b[n - 1]) / d[n - 2];
    for (int i = n - 3; i >= 0; --i) b[i] = (b[i] - du[i] * b[i + 1] - du2[i] * b[i + 2]) / d[i];
}

// Eigenpairs of (T - iτE_1) v = μ D v on n nodes (1D absorbing T of Theorem A.2).
static int mean_eigen(int n, double h, double kbar, std::vector<cplx>& mu, std::vector<cplx>& V,
                      double* cond_out = nullptr) {
    const double ih2 = 1.0 / (h * h), tau = kbar / h;
    std::vector<double> dw(n, 1.0);
    dw[0] = dw[n - 1] = 0.5;
    // J = D^{-1/2} (T - iτE_1) D^{-1/2}
    std::vector<cplx> jd(n), je(n - 1);
    for (int i = 0; i < n; ++i) {
        double t = (i == 0 || i == n - 1) ? ih2 : 2.0 * ih2;
        cplx v = t;
        if (i == 0 || i == n - 1) v -= cplx(0.0, tau);
        jd[i] = v / dw[i];
    }
    for (int i = 0; i < n - 1; ++i) je[i] = -ih2 / std::sqrt(dw[i] * dw[i + 1]);
    mu = jd;
    if (!ql_eigenvalues(mu, je)) return fail(SG_ESETUP, "QL eigenvalue iteration did not converge");
    std::sort(mu.begin(), mu.end(), [](cplx a, cplx b) { return a.real() < b.real(); });
    // eigenvectors of J by inverse iteration with a slightly perturbed shift
    V.assign((size_t)n * n, 0.0);
    double jnorm = 4.0 * ih2 + 2.0 * tau;
    std::vector<cplx> dl, dd, du, du2, u(n);
    std::vector<uint8_t> piv;
    for (int a = 0; a < n; ++a) {
        cplx sh = mu[a] + cplx(1e-13, 1e-13) * jnorm;
        dl.assign(je.begin(), je.end());
        du.assign(je.begin(), je.end());
        dd.resize(n);
        for (int i = 0; i < n; ++i) dd[i] = jd[i] - sh;
        if (!tri_lu(n, dl, dd, du, du2, piv)) return fail(SG_ESETUP, "singular shifted eigen system");
        for (int i = 0; i < n; ++i) u[i] = 1.0 + 0.37 * std::sin(1.0 + 7.13 * i) + cplx(0, 0.11 * std::cos(3.1 * i));
        for (int it = 0; it < 3; ++it) {
            tri_solve(n, dl, dd, du, du2, piv, u);
            double nr = 0;
            for (auto& z : u) nr += std::norm(z);
            nr = std::sqrt(nr);
            for (auto& z : u) z /= nr;
        }
        cplx uu = 0;
        for (auto& z : u) uu += z * z;
        // refine the eigenvalue by the (unconjugated) Rayleigh quotient uᵀJu / uᵀu, which is
        // second-order accurate for the complex symmetric J
        cplx uju = 0;
        for (int i = 0; i < n; ++i) {
            cplx ju = jd[i] * u[i];
            if (i > 0) ju += je[i - 1] * u[i - 1];
            if (i < n - 1) ju += je[i] * u[i + 1];
            uju += u[i] * ju;
        }
        mu[a] = uju / uu;
        cplx sc = 1.0 / std::sqrt(uu);
        for (int i = 0; i < n; ++i) V[(size_t)i * n + a] = u[i] * sc / std::sqrt(dw[i]);
    }
    // validation: residual and D-orthonormality of the eigenvectors
    double vmax = 0, res = 0;
    for (size_t i = 0; i < V.size(); ++i) vmax = std::max(vmax, std::abs(V[i]));
    for (int a = 0; a < n; ++a) {
        for (int i = 0; i < n; ++i) {
            double t = (i == 0 || i == n - 1) ? ih2 : 2.0 * ih2;
            cplx Tv = t * V[(size_t)i * n + a];
            if (i > 0) Tv -= ih2 * V[(size_t)(i - 1) * n + a];
            if (i < n - 1) Tv -= ih2 * V[(size_t)(i + 1) * n + a];
            if (i == 0 || i == n - 1) Tv -= cplx(0, tau) * V[(size_t)i * n + a];
            cplx r = Tv - mu[a] * dw[i] * V[(size_t)i * n + a];
            res = std::max(res, std::abs(r));
        }
    }
    res /= (jnorm * vmax);
    double orth = 0;
    for (int a = 0; a < n; ++a)
        for (int b = a; b < n; ++b) {
            cplx acc = 0;
            for (int i = 0; i < n; ++i) acc += V[(size_t)i * n + a] * dw[i] * V[(size_t)i * n + b];
            orth = std::max(orth, std::abs(acc - (a == b ? 1.0 : 0.0)));
        }
    // condition of the eigenvector matrix: Ṽ^{-1} = Ṽᵀ D, so cond₂(Ṽ) = ||Ṽ||₂ ||Ṽᵀ D||₂ (the
    // block solve's rounding grows like cond₂(Ṽ)²).  The Frobenius norms bound it cheaply;
    // only when that bound exceeds 1e3 are the two 2-norms estimated by power iteration.
    if (cond_out) {
        double fa = 0, fb = 0;
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) {
                fa += std::norm(V[(size_t)i * n + k]);
                fb += std::norm(V[(size_t)i * n + k] * dw[i]);
            }
        double cond = std::sqrt(fa * fb);
        if (cond > 1e3) {
            auto norm2 = [&](bool inverse) {   // M = Ṽ or Ṽᵀ D: sqrt of the top eigenvalue of MᴴM
                std::vector<cplx> u(n), t(n);
                for (int i = 0; i < n; ++i) u[i] = cplx(1.0 + 0.1 * std::sin(0.7 * i), 0.05 * std::cos(1.3 * i));
                double lam = 0;
                for (int it = 0; it < 30; ++it) {
                    double nr = 0;
                    for (auto& z : u) nr += std::norm(z);
                    nr = std::sqrt(nr);
                    for (auto& z : u) z /= nr;
                    for (int i = 0; i < n; ++i) {
                        cplx acc = 0;
                        for (int k = 0; k < n; ++k)
                            acc += (inverse ? V[(size_t)k * n + i] * dw[k] : V[(size_t)i * n + k]) * u[k];
                        t[i] = acc;
                    }
                    for (int k = 0; k < n; ++k) {
                        cplx acc = 0;
                        for (int i = 0; i < n; ++i)
                            acc += std::conj(inverse ? V[(size_t)k * n + i] * dw[k] : V[(size_t)i * n + k]) * t[i];
                        u[k] = acc;
                    }
                    double un = 0;
                    for (auto& z : u) un += std::norm(z);
                    lam = std::sqrt(un);
                }
                return std::sqrt(lam);
            };
            cond = norm2(false) * norm2(true);
        }
        *cond_out = cond;
    }
    if (!(res < 1e-10) || !(orth < 1e-8))
    {
        char msg[160];
        std::snprintf(msg, sizeof msg, "eigenfactor validation failed: residual %.3e, D-orthonormality defect %.3e", res,
                      orth);
        return fail(SG_ESETUP, msg);
    }
    return SG_OK;
}

// Factors of (T - iτE_1 + σ_a D) for the systems a (1D absorbing T), uploaded row-major.
static int build_tri(int n, double h, double kbar, const std::vector<cplx>& sig, TriFactors& tf) {
    const int nsys = (int)sig.size();
    const double ih2 = 1.0 / (h * h), tau = kbar / h;
    std::vector<double2> hdl((size_t)std::max(n - 1, 1) * nsys), hdi((size_t)n * nsys),
        hu1((size_t)std::max(n - 1, 1) * nsys), hu2((size_t)std::max(n - 2, 1) * nsys);
    std::vector<uint8_t> hp((size_t)std::max(n - 1, 1) * nsys);
    std::vector<cplx> dl, d, du, du2;
    std::vector<uint8_t> piv;
    for (int a = 0; a < nsys; ++a) {
        dl.assign(n - 1, -ih2);
        du.assign(n - 1, -ih2);
        d.resize(n);
        for (int i = 0; i < n; ++i) {
            bool bnd = (i == 0 || i == n - 1);
            d[i] = (bnd ? ih2 : 2.0 * ih2) + sig[a] * (bnd ? 0.5 : 1.0);
            if (bnd) d[i] -= cplx(0, tau);
        }
        if (!tri_lu(n, dl, d, du, du2, piv)) return fail(SG_ESETUP, "singular mean-block tridiagonal system");
        for (int i = 0; i < n; ++i) {
            cplx inv = 1.0 / d[i];
            hdi[(size_t)i * nsys + a] = make_double2(inv.real(), inv.imag());
        }
        for (int i = 0; i < n - 1; ++i) {
            hdl[(size_t)i * nsys + a] = make_double2(dl[i].real(), dl[i].imag());
            hu1[(size_t)i * nsys + a] = make_double2(du[i].real(), du[i].imag());
            hp[(size_t)i * nsys + a] = piv[i];
        }
        for (int i = 0; i < n - 2; ++i) hu2[(size_t)i * nsys + a] = make_double2(du2[i].real(), du2[i].imag());
    }
    tf.len = n;
    tf.nsys = nsys;
    // Segmented form of the two substitutions: with K segments of L rows, the forward
    // carried value obeys c_{i+1} = A_i c_i + B_i b_{i+1} (A_i = 1 after a row exchange,
    // -l_i otherwise), the backward one X_i = M_i X_{i+1} + (y_i/u_ii, 0) with
    // M_i = [[-u_{i,i+1}/u_ii, -u_{i,i+2}/u_ii], [1, 0]]; the products of A_i and of M_i over
    // each segment are the propagators used to join independently computed segments.
    int K = 1;
    while (K < 32 && (n + K - 1) / K > 8) K *= 2;
    const int L = (n + K - 1) / K;
    tf.K = K;
    tf.L = L;
    std::vector<double2> hu1p((size_t)n * nsys, make_double2(0, 0)), hu2p((size_t)n * nsys, make_double2(0, 0));
    std::vector<double2> hphi((size_t)K * nsys), hpsi((size_t)K * nsys * 4);
    std::vector<uint32_t> hpm((size_t)K * nsys, 0u);
    for (int a = 0; a < nsys; ++a) {
        auto C = [&](const std::vector<double2>& v, size_t idx) { return cplx(v[idx].x, v[idx].y); };
        for (int i = 0; i < n; ++i) {
            const cplx di = C(hdi, (size_t)i * nsys + a);
            if (i < n - 1) {
                const cplx u1 = C(hu1, (size_t)i * nsys + a) * di;
                hu1p[(size_t)i * nsys + a] = make_double2(u1.real(), u1.imag());
            }
            if (i < n - 2) {
                const cplx u2 = C(hu2, (size_t)i * nsys + a) * di;
                hu2p[(size_t)i * nsys + a] = make_double2(u2.real(), u2.imag());
            }
        }
        for (int k = 0; k < K; ++k) {
            const int s0 = k * L, e0 = std::min(s0 + L, n);
            cplx ph = 1.0;
            for (int i = s0; i < e0 && i <= n - 2; ++i)
                ph *= hp[(size_t)i * nsys + a] ? cplx(1.0) : -C(hdl, (size_t)i * nsys + a);
            hphi[(size_t)k * nsys + a] = make_double2(ph.real(), ph.imag());
            uint32_t bits = 0;
            for (int i = s0; i < e0 && i <= n - 2; ++i)
                if (hp[(size_t)i * nsys + a]) bits |= 1u << (i - s0);
            hpm[(size_t)k * nsys + a] = bits;
            cplx m00 = 1.0, m01 = 0.0, m10 = 0.0, m11 = 1.0;   // product M_s ... M_{e-1}
            for (int i = e0 - 1; i >= s0; --i) {
                const cplx u1 = C(hu1p, (size_t)i * nsys + a), u2 = C(hu2p, (size_t)i * nsys + a);
                // left-multiply by M_i = [[-u1, -u2], [1, 0]]
                const cplx n00 = -u1 * m00 - u2 * m10, n01 = -u1 * m01 - u2 * m11;
                const cplx n10 = m00, n11 = m01;
                m00 = n00; m01 = n01; m10 = n10; m11 = n11;
            }
            const size_t o = ((size_t)k * nsys + a) * 4;
            hpsi[o + 0] = make_double2(m00.real(), m00.imag());
            hpsi[o + 1] = make_double2(m01.real(), m01.imag());
            hpsi[o + 2] = make_double2(m10.real(), m10.imag());
            hpsi[o + 3] = make_double2(m11.real(), m11.imag());
        }
    }
    SG_HIP(setup_alloc(&tf.u1p, hu1p.size() * sizeof(double2)));
    SG_HIP(setup_alloc(&tf.u2p, hu2p.size() * sizeof(double2)));
    SG_HIP(setup_alloc(&tf.phi, hphi.size() * sizeof(double2)));
    SG_HIP(setup_alloc(&tf.psi, hpsi.size() * sizeof(double2)));
    if (int rc_ = upload(tf.u1p, hu1p.data(), hu1p.size() * sizeof(double2))) return rc_;
    if (int rc_ = upload(tf.u2p, hu2p.data(), hu2p.size() * sizeof(double2))) return rc_;
    if (int rc_ = upload(tf.phi, hphi.data(), hphi.size() * sizeof(double2))) return rc_;
    if (int rc_ = upload(tf.psi, hpsi.data(), hpsi.size() * sizeof(double2))) return rc_;
    SG_HIP(setup_alloc(&tf.pivm, hpm.size() * sizeof(uint32_t)));
    if (int rc_ = upload(tf.pivm, hpm.data(), hpm.size() * sizeof(uint32_t))) return rc_;
    SG_HIP(setup_alloc(&tf.dl, hdl.size() * sizeof(double2)));
    SG_HIP(setup_alloc(&tf.dinv, hdi.size() * sizeof(double2)));
    SG_HIP(setup_alloc(&tf.du1, hu1.size() * sizeof(double2)));
    SG_HIP(setup_alloc(&tf.du2, hu2.size() * sizeof(double2)));
    SG_HIP(setup_alloc(&tf.piv, hp.size()));
    if (int rc_ = upload(tf.dl, hdl.data(), hdl.size() * sizeof(double2))) return rc_;
    if (int rc_ = upload(tf.dinv, hdi.data(), hdi.size() * sizeof(double2))) return rc_;
    if (int rc_ = upload(tf.du1, hu1.data(), hu1.size() * sizeof(double2))) return rc_;
    if (int rc_ = upload(tf.du2, hu2.data(), hu2.size() * sizeof(double2))) return rc_;
    if (int rc_ = upload(tf.piv, hp.data(), hp.size())) return rc_;
    return SG_OK;
}

static void free_tri(TriFactors& t) {
    (void)hipFree(t.dl);
    (void)hipFree(t.dinv);
    (void)hipFree(t.du1);
    (void)hipFree(t.du2);
    (void)hipFree(t.piv);
    (void)hipFree(t.u1p);
    (void)hipFree(t.u2p);
    (void)hipFree(t.phi);
    (void)hipFree(t.psi);
    (void)hipFree(t.pivm);
    t = TriFactors{};
}

Ctx::~Ctx() {
    (void)hipFree(d_D2);
    (void)hipFree(d_D1);
    (void)hipFree(d_prog);
    (void)hipFree(d_vals);
    (void)hipFree(d_w);
    (void)hipFree(d_kf);
    (void)hipFree(fwd.f64);
    (void)hipFree(fwd.f32);
    (void)hipFree(fwd.bf_hi);
    (void)hipFree(fwd.bf_lo);
    (void)hipFree(inv.f64);
    (void)hipFree(inv.f32);
    (void)hipFree(inv.bf_hi);
    (void)hipFree(inv.bf_lo);
    (void)hipFree(fwd.p3);
    (void)hipFree(inv.p3);
    (void)hipFree(fwd.p3f);
    (void)hipFree(inv.p3f);
    for (auto& t : tri) free_tri(t);
    (void)hipFree(ws.V);
    (void)hipFree(ws.Z);
    (void)hipFree(ws.tmp);
    (void)hipFree(ws.scale);
    (void)hipFree(ws.coef);
    (void)hipFree(ws.partial);
    if (ws.host_pinned) (void)hipHostFree(ws.host_pinned);
    if (ws.done) (void)hipEventDestroy(ws.done);
    (void)hipFree(ws.dpart);
    (void)hipFree(ws.dsmall);
    if (ws.hrec) (void)hipHostFree(ws.hrec);
    (void)hipFree(d_tmp_pc);
    (void)hipFree(d_k0);
    (void)hipFree(d_lineE[0]);
    (void)hipFree(d_lineE[1]);
    (void)hipFree(d_lineb);
}

// ------------------------------------------------------------------ setup

static std::atomic<double> g_eigen_cond_limit{1e4};
double eigen_cond_limit() { return g_eigen_cond_limit.load(); }
void set_eigen_cond_limit(double v) { g_eigen_cond_limit.store(v); }

static thread_local hipStream_t t_setup_stream = nullptr;
static thread_local SetupClock t_setup_clock;

static double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

SetupClock& setup_clock() { return t_setup_clock; }

static void stamp_setup(Ctx* c, std::chrono::steady_clock::time_point t0) {
    c->t_setup_ms = ms_since(t0);
    c->t_setup_alloc_ms = t_setup_clock.alloc;
    c->t_setup_upload_ms = t_setup_clock.upload;
    c->t_setup_stream_ms = t_setup_clock.stream;
}

hipError_t setup_alloc_raw(void** p, size_t bytes) {
    const auto t0 = std::chrono::steady_clock::now();
    const hipError_t e = hipMalloc(p, bytes);
    t_setup_clock.alloc += ms_since(t0);
    return e;
}

SetupStream::SetupStream() {
    rc = SG_OK;
    t_setup_clock = SetupClock{};
    const auto t0 = std::chrono::steady_clock::now();
    if (hipStreamCreateWithFlags(&t_setup_stream, hipStreamNonBlocking) != hipSuccess) {
        t_setup_stream = nullptr;
        rc = fail(SG_EHIP, "could not create the setup stream");
    }
    t_setup_clock.stream += ms_since(t0);
}
SetupStream::~SetupStream() {
    if (t_setup_stream) (void)hipStreamDestroy(t_setup_stream);
    t_setup_stream = nullptr;
}

int upload(void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return SG_OK;
    const auto t0 = std::chrono::steady_clock::now();
    SG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, t_setup_stream));
    SG_HIP(hipStreamSynchronize(t_setup_stream));   // src may be freed when this returns
    t_setup_clock.upload += ms_since(t0);
    return SG_OK;
}

int upload_zero(void* dst, size_t bytes) {
    if (bytes == 0) return SG_OK;
    SG_HIP(hipMemsetAsync(dst, 0, bytes, t_setup_stream));
    SG_HIP(hipStreamSynchronize(t_setup_stream));
    return SG_OK;
}

int build_ctx(const sg_problem* p, hipStream_t stream, Ctx** out) {
    auto t0 = std::chrono::steady_clock::now();
    SetupStream setup_stream;
    if (setup_stream.rc) return setup_stream.rc;
    if (!p || !out) return fail(SG_EINVAL, "null argument");
    if (p->dim != 1 && p->dim != 2) return fail(SG_EINVAL, "dim must be 1 or 2");
    if (p->bc != SG_BC_ABSORBING) return fail(SG_EINVAL, "only absorbing boundary conditions are supported");
    if (p->n < 3 || p->n > 8192) return fail(SG_EINVAL, "n must be in [3, 8192]");
    if (p->s < 1 || p->s > 8 || p->degree < 0 || p->degree > 8)
        return fail(SG_EINVAL, "need 1 <= s <= 8 and 0 <= degree <= 8");
    if (!p->k_fields) return fail(SG_EINVAL, "k_fields is null");
    std::unique_ptr<Ctx> c(new Ctx());
    SG_HIP(hipGetDevice(&c->device));
    c->dim = p->dim;
    c->n = p->n;
    c->s = p->s;
    c->degree = p->degree;
    c->h = 1.0 / (p->n - 1);
    c->kbar = p->k_mean;
    c->beta = p->csl_beta;
    c->P = 1;
    for (int d = 0; d < p->dim; ++d) c->P *= p->n;
    const long long P = c->P;
    const int s = p->s;
    if (p->k_mean == 0.0) {
        // spatially varying mean (Section 7): exact line block LU instead of fast diagonalisation
        c->vmean = true;
        if (p->dim == 2 && p->n > 257)
            return fail(SG_EINVAL, "a spatially varying mean needs n <= 257 in 2D (its line factorisation costs O(n^4) on the host)");
        for (long long i = 0; i < P; ++i)
            if (!std::isfinite(p->k_fields[i])) return fail(SG_EINVAL, "k_0 must be finite");
    } else {
        for (long long i = 0; i < P; ++i)
            if (p->k_fields[i] != p->k_mean)
                return fail(SG_EINVAL, "k_0 must be spatially constant and equal to k_mean (or k_mean = 0 for a "
                                       "spatially varying mean)");
        if (!(p->k_mean > 0)) return fail(SG_EINVAL, "k_mean must be positive");
    }

    c->alpha = make_basis(s, p->degree);
    c->Q = (int)(c->alpha.size() / s);
    c->nvec = (long long)c->Q * P;
    const int Q = c->Q;

    // fields of k (degree <= 1) and k² (degree <= 2) in the Ψ_γ basis
    auto unit = [&](int l) { std::vector<int> g(s, 0); g[l] = 1; return g; };
    c->gamma1.push_back(std::vector<int>(s, 0));
    for (int l = 0; l < s; ++l) c->gamma1.push_back(unit(l));
    c->gamma2 = c->gamma1;
    for (int l = 0; l < s; ++l) { auto g = std::vector<int>(s, 0); g[l] = 2; c->gamma2.push_back(g); }
    for (int l = 0; l < s; ++l)
        for (int m = l + 1; m < s; ++m) { auto g = std::vector<int>(s, 0); g[l] = 1; g[m] = 1; c->gamma2.push_back(g); }
    build_coupling(c->alpha, Q, s, c->gamma2, c->K);
    build_coupling(c->alpha, Q, s, c->gamma1, c->B);
    // a shape that neither a specialised operator kernel nor the generic one (whose LDS tile
    // grows with Q) can serve is refused here rather than at the first sg_apply
    if (!apply_available(c.get(), 0.0))
        return fail(SG_EINVAL, "no operator kernel serves this (dim, s, degree): Q = " + std::to_string(Q) +
                                   " is too large for the generic kernel's LDS tile");

    const int n = p->n;
    std::vector<double> dw(n, 1.0);
    dw[0] = dw[n - 1] = 0.5;
    std::vector<double> w(P), e(P);
    for (long long idx = 0; idx < P; ++idx) {
        if (p->dim == 1) {
            w[idx] = dw[idx];
            e[idx] = (idx == 0 || idx == n - 1) ? 1.0 : 0.0;
        } else {
            int i = (int)(idx % n), j = (int)(idx / n);
            w[idx] = dw[i] * dw[j];
            e[idx] = (i == 0 || j == 0 || i == n - 1 || j == n - 1) ? 1.0 : 0.0;
        }
    }
    const int ng1 = (int)c->gamma1.size(), ng2 = (int)c->gamma2.size();
    std::vector<double> D1((size_t)ng1 * P), D2((size_t)ng2 * P);
    const double r3 = std::sqrt(3.0), r5 = std::sqrt(5.0);
    for (long long idx = 0; idx < P; ++idx) {
        const double k0 = p->k_fields[idx];
        double sumsq = 0;
        for (int l = 0; l < s; ++l) { double kl = p->k_fields[(size_t)(l + 1) * P + idx]; sumsq += kl * kl; }
        int g = 0;
        D2[(size_t)g * P + idx] = w[idx] * (k0 * k0 + sumsq / 3.0);
        D1[(size_t)g * P + idx] = e[idx] / c->h * k0;
        ++g;
        for (int l = 0; l < s; ++l, ++g) {
            double kl = p->k_fields[(size_t)(l + 1) * P + idx];
            D2[(size_t)g * P + idx] = w[idx] * 2.0 * k0 * kl / r3;
            D1[(size_t)g * P + idx] = e[idx] / c->h * kl / r3;
        }
        for (int l = 0; l < s; ++l, ++g) {
            double kl = p->k_fields[(size_t)(l + 1) * P + idx];
            D2[(size_t)g * P + idx] = w[idx] * 2.0 * kl * kl / (3.0 * r5);
        }
        for (int l = 0; l < s; ++l)
            for (int m = l + 1; m < s; ++m, ++g) {
                double kl = p->k_fields[(size_t)(l + 1) * P + idx];
                double km = p->k_fields[(size_t)(m + 1) * P + idx];
                D2[(size_t)g * P + idx] = w[idx] * 2.0 * kl * km / 3.0;
            }
    }

    // packed integer program: K tables, B tables, output order (heaviest outputs first)
    std::vector<int> prog;
    auto put = [&](const std::vector<int>& v) { int off = (int)prog.size(); prog.insert(prog.end(), v.begin(), v.end()); return off; };
    c->kprog_pairptr = put(c->K.pair_ptr);
    c->kprog_pairj = put(c->K.pair_j);
    c->kprog_termptr = put(c->K.term_ptr);
    c->kprog_termfield = put(c->K.term_field);
    c->bprog_pairptr = put(c->B.pair_ptr);
    c->bprog_pairj = put(c->B.pair_j);
    c->bprog_termptr = put(c->B.term_ptr);
    c->bprog_termfield = put(c->B.term_field);
    std::vector<int> order(Q);
    for (int i = 0; i < Q; ++i) order[i] = i;
    c->out_order_off = put(order);
    std::vector<double> vals(c->K.term_val);
    c->kvals_off = 0;
    c->bvals_off = (int)vals.size();
    vals.insert(vals.end(), c->B.term_val.begin(), c->B.term_val.end());

    SG_HIP(setup_alloc(&c->d_D2, D2.size() * sizeof(double)));
    SG_HIP(setup_alloc(&c->d_D1, D1.size() * sizeof(double)));
    SG_HIP(setup_alloc(&c->d_prog, prog.size() * sizeof(int)));
    SG_HIP(setup_alloc(&c->d_vals, std::max<size_t>(vals.size(), 1) * sizeof(double)));
    SG_HIP(setup_alloc(&c->d_w, w.size() * sizeof(double)));
    if (int rc_ = upload(c->d_D2, D2.data(), D2.size() * sizeof(double))) return rc_;
    if (int rc_ = upload(c->d_D1, D1.data(), D1.size() * sizeof(double))) return rc_;
    if (int rc_ = upload(c->d_prog, prog.data(), prog.size() * sizeof(int))) return rc_;
    if (!vals.empty())
        if (int rc_ = upload(c->d_vals, vals.data(), vals.size() * sizeof(double))) return rc_;
    if (int rc_ = upload(c->d_w, w.data(), w.size() * sizeof(double))) return rc_;
    c->w_host = w;
    SG_HIP(setup_alloc(&c->d_kf, (size_t)s * P * sizeof(double)));
    if (int rc_ = upload(c->d_kf, p->k_fields + P, (size_t)s * P * sizeof(double))) return rc_;

    if (c->vmean) {
        SG_HIP(setup_alloc(&c->d_k0, (size_t)P * sizeof(double)));
        if (int rc_ = upload(c->d_k0, p->k_fields, (size_t)P * sizeof(double))) return rc_;
        int rc = build_line_factors(c.get(), p->k_fields);
        if (rc) return rc;
        stamp_setup(c.get(), t0);
        *out = c.release();
        return SG_OK;
    }
    // mean-block factors for A_0 (c = k̄²) and M_0 (c = (1+iβ)k̄²)
    const double kb = p->k_mean;
    const cplx cshift[2] = {cplx(kb * kb, 0.0), cplx(kb * kb, p->csl_beta * kb * kb)};
    if (p->dim == 1) {
        for (int t = 0; t < 2; ++t) {
            std::vector<cplx> sig(1, -cshift[t]);
            int rc = build_tri(n, c->h, kb, sig, c->tri[t]);
            if (rc) return rc;
        }
    } else {
        int rc = mean_eigen(n, c->h, kb, c->mu, c->Vt, &c->cond_v);
        if (rc == SG_OK && !(c->cond_v <= eigen_cond_limit()))
            rc = fail(SG_ESETUP, "eigenvector matrix of the mean block too ill-conditioned: cond " +
                                     std::to_string(c->cond_v));
        if (rc == SG_ESETUP && n <= 257) {
            // fall back to the exact line factorisation of the same (constant-k̄) mean block,
            // the paper's own approach of factorising the block (Section 6.3)
            c->vmean = true;
            c->eig_fallback = true;
            std::vector<double> k0(P, kb);
            rc = build_line_factors(c.get(), k0.data());
            if (rc) return rc;
            stamp_setup(c.get(), t0);
            *out = c.release();
            return SG_OK;
        }
        if (rc) return rc;
        for (int t = 0; t < 2; ++t) {
            std::vector<cplx> sig(n);
            for (int a = 0; a < n; ++a) sig[a] = c->mu[a] - cshift[t];
            rc = build_tri(n, c->h, kb, sig, c->tri[t]);
            if (rc) return rc;
        }
        rc = upload_dense_b(c.get(), stream);
        if (rc) return rc;
    }
    // rows of the intermediate start on 128-byte boundaries, so that the sweep's and the
    // transforms' row pieces are whole cache lines
    c->tld = c->dim == 2 ? (n + 7) / 8 * 8 : n;
    SG_HIP(setup_alloc(&c->d_tmp_pc, (c->dim == 2 ? (size_t)c->Q * n * c->tld : (size_t)c->nvec) * sizeof(double2)));
    stamp_setup(c.get(), t0);
    *out = c.release();
    return SG_OK;
}

}  // namespace sgi
