"""Statistics of the stochastic Galerkin solution (Section 7, Figures bE_Var and
k123_convergence).

The SG approximation is u_m(x, ξ) = Σ_i V_i(x) φ_i(ξ) (eq. Galerkin_approx, vector
V = [V_0; ...; V_m], eq. LGS_from_FD_G).  These functions evaluate its statistics by their
definitions, with no use of the orthonormality of the basis: the expectation over
ξ ~ U[-1,1]^s is a tensor Gauss-Legendre quadrature of the polynomial u_m, exact for the
degrees involved (2r+1 nodes per variable integrate the squares of degree-r polynomials).

expectation      E[u_m](x) = ∫ u_m(x, ξ) ρ(ξ) dξ
variance_re_im   Var[Re u_m](x), Var[Im u_m](x)  (the real and imaginary parts, as plotted)
degree_magnitudes  γ_j = max{ ||V_i||_∞ : deg φ_i = j }, j = 0..r  (eq. magnitude_V)
"""
from __future__ import annotations

import itertools

import numpy as np

from .pc import multi_indices, orthonormal_legendre


def _quadrature(s: int, r: int):
    """Nodes (npts × s) and weights (npts) of the tensor Gauss-Legendre rule for the
    uniform density 2^{-s} on [-1,1]^s, exact for polynomials of degree 4r+1 in each
    variable."""
    g, w = np.polynomial.legendre.leggauss(2 * r + 1)
    nodes = np.array(list(itertools.product(g, repeat=s)))
    weights = np.array([np.prod(t) for t in itertools.product(w / 2.0, repeat=s)])
    return nodes, weights


def _basis_at(s: int, r: int, nodes: np.ndarray) -> np.ndarray:
    """φ_i(ξ_q) for every basis index i and quadrature node q: (Q × npts)."""
    alpha = multi_indices(s, r)
    phi1 = [orthonormal_legendre(r, nodes[:, l]) for l in range(s)]   # (r+1) × npts each
    out = np.ones((alpha.shape[0], nodes.shape[0]))
    for i, a in enumerate(alpha):
        for l in range(s):
            out[i] *= phi1[l][a[l]]
    return out


def _samples(V: np.ndarray, s: int, r: int, P: int):
    nodes, weights = _quadrature(s, r)
    B = _basis_at(s, r, nodes)
    Vm = np.asarray(V, dtype=np.complex128).reshape(B.shape[0], P)
    U = B.T @ Vm          # u_m(x, ξ_q): npts × P
    return U, weights


def expectation(V: np.ndarray, s: int, r: int, P: int) -> np.ndarray:
    """E[u_m] at the P nodes (complex)."""
    U, w = _samples(V, s, r, P)
    return w @ U


def variance_re_im(V: np.ndarray, s: int, r: int, P: int):
    """(Var[Re u_m], Var[Im u_m]) at the P nodes."""
    U, w = _samples(V, s, r, P)
    mean = w @ U
    vr = w @ (U.real - mean.real) ** 2
    vi = w @ (U.imag - mean.imag) ** 2
    return vr, vi


def degree_magnitudes(V: np.ndarray, s: int, r: int, P: int) -> np.ndarray:
    """γ_j = max over the basis polynomials of total degree exactly j of ||V_i||_∞."""
    alpha = multi_indices(s, r)
    Vm = np.asarray(V, dtype=np.complex128).reshape(alpha.shape[0], P)
    deg = alpha.sum(axis=1)
    return np.array([np.max(np.abs(Vm[deg == j])) for j in range(r + 1)])
