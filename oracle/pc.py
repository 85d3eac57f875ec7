"""Polynomial chaos basis and Galerkin moment tables (Section 2.3, Section 3.2).

The basis is the set of products of univariate orthonormal Legendre
polynomials of total degree <= r in s uniform random variables ξ_ℓ ~ U[-1,1],
with density ρ = 2^-s on [-1,1]^s (Section 2.2) and φ_0 ≡ 1.  Its size is
m+1 = (s+r)!/(s! r!) (eq. number_basis_polynomial).

The Galerkin entries needed by the assembly are moments E[ξ_a ξ_b φ_i φ_j]
(ξ_0 ≡ 1), computed here by Gauss-Legendre quadrature of the univariate
factors.  Entries that are zero in exact arithmetic come out at roundoff level;
they are set to exactly zero (|x| < 1e-13) and the tables are symmetrised, so
that the assembled matrix is exactly complex symmetric and its nonzero count
is the exact-arithmetic one (Table construct_A).

Multi-index order (the paper leaves it open): graded by total degree, and
within one degree lexicographically descending, e.g. for s=2:
(0,0), (1,0), (0,1), (2,0), (1,1), (0,2).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

ZERO_THRESHOLD = 1e-13


def basis_size(s: int, r: int) -> int:
    """m+1 = (s+r)!/(s! r!) (eq. number_basis_polynomial)."""
    return math.comb(s + r, s)


def multi_indices(s: int, r: int) -> np.ndarray:
    """All α ∈ N_0^s with |α| <= r, graded, descending-lexicographic per degree."""
    out = []
    for d in range(r + 1):
        level = [a for a in itertools.product(range(d + 1), repeat=s) if sum(a) == d]
        level.sort(reverse=True)
        out.extend(level)
    return np.array(out, dtype=np.int64).reshape(len(out), s)


def orthonormal_legendre(nmax: int, x: np.ndarray) -> np.ndarray:
    """Values φ_0..φ_nmax at x, φ_n = sqrt(2n+1) P_n (orthonormal for density 1/2).

    P_n from Bonnet's recurrence (n+1)P_{n+1} = (2n+1) x P_n - n P_{n-1}.
    """
    x = np.asarray(x, dtype=np.float64)
    P = np.zeros((nmax + 1,) + x.shape)
    P[0] = 1.0
    if nmax >= 1:
        P[1] = x
    for n in range(1, nmax):
        P[n + 1] = ((2 * n + 1) * x * P[n] - n * P[n - 1]) / (n + 1)
    scale = np.sqrt(2.0 * np.arange(nmax + 1) + 1.0)
    return P * scale.reshape((-1,) + (1,) * x.ndim)


def univariate_moments(nmax: int, pmax: int = 2) -> np.ndarray:
    """M[p, a, b] = E[ξ^p φ_a(ξ) φ_b(ξ)] for ξ ~ U[-1,1], p <= pmax, a,b <= nmax.

    Gauss-Legendre with nmax + pmax//2 + 2 nodes integrates degree <= 2nmax+pmax exactly.
    """
    nodes, weights = np.polynomial.legendre.leggauss(nmax + pmax // 2 + 2)
    weights = weights / 2.0  # density 1/2 on [-1,1]
    phi = orthonormal_legendre(nmax, nodes)
    M = np.empty((pmax + 1, nmax + 1, nmax + 1))
    for p in range(pmax + 1):
        M[p] = (phi * (weights * nodes ** p)) @ phi.T
    return M


def _clean(T: np.ndarray) -> np.ndarray:
    T = np.where(np.abs(T) < ZERO_THRESHOLD, 0.0, T)
    return 0.5 * (T + T.T)


def moment_tables(s: int, r: int) -> np.ndarray:
    """E[a, b, i, j] = E[ξ_a ξ_b φ_i φ_j] for a, b ∈ {0..s} (ξ_0 ≡ 1).

    The multivariate φ_i = Π_ℓ φ_{α_iℓ}(ξ_ℓ) and independence of the ξ_ℓ make each
    moment a product of univariate moments with exponent p_ℓ = [a=ℓ] + [b=ℓ].
    """
    alpha = multi_indices(s, r)
    Q = alpha.shape[0]
    M = univariate_moments(r, 2)
    E = np.zeros((s + 1, s + 1, Q, Q))
    for a in range(s + 1):
        for b in range(a, s + 1):
            T = np.ones((Q, Q))
            for l in range(s):
                p = int(a == l + 1) + int(b == l + 1)
                T *= M[p][np.ix_(alpha[:, l], alpha[:, l])]
            T = _clean(T)
            E[a, b] = T
            E[b, a] = T
    return E


def k_coupling(k_fields: np.ndarray, E: np.ndarray):
    """Per-node Galerkin coupling weights of k and k² (eqs. b_ij and c_ij).

    Returns (B, C) as lists of (table, field) terms with
      b_ij(x) = Σ_a k_a(x) E[ξ_a φ_i φ_j],
      c_ij(x) = Σ_{a,b} k_a(x) k_b(x) E[ξ_a ξ_b φ_i φ_j],
    written through the monomial expansion of k and k² in ξ.
    """
    s1 = k_fields.shape[0]
    B = [(E[a, 0], k_fields[a]) for a in range(s1)]
    C = []
    for a in range(s1):
        for b in range(a, s1):
            mult = 1.0 if a == b else 2.0
            C.append((E[a, b], mult * k_fields[a] * k_fields[b]))
    return B, C
