"""Finite-difference building blocks (Appendix A).

Nodes are x_i = i·h.  Absorbing BC uses nodes i = 0..q+1 (n = q+2) with
h = 1/(q+1); Dirichlet BC keeps the interior nodes i = 1..q only (n = q).
2D vectors are ordered x fastest (Theorem A.3): flat index j·n + i for node
(x_i, y_j), so kron(A, B) applies A along y and B along x.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def T_absorbing(n: int, h: float) -> sp.csr_matrix:
    """Theorem A.2, matrix T: (1/h²) tridiag(-1, 2, -1) with corner entries 1/h²."""
    main = np.full(n, 2.0)
    main[0] = main[-1] = 1.0
    off = -np.ones(n - 1)
    return (sp.diags([off, main, off], [-1, 0, 1], format="csr") / (h * h)).tocsr()


def T_dirichlet(q: int, h: float) -> sp.csr_matrix:
    """Theorem A.1, matrix T: (1/h²) tridiag(-1, 2, -1) on the q interior nodes."""
    main = np.full(q, 2.0)
    off = -np.ones(q - 1)
    return (sp.diags([off, main, off], [-1, 0, 1], format="csr") / (h * h)).tocsr()


def half_weights(n: int) -> np.ndarray:
    """D = diag(1/2, 1, ..., 1, 1/2) (Theorem A.2 D_2 weights, Theorem A.4 matrix D)."""
    d = np.ones(n)
    d[0] = d[-1] = 0.5
    return d


def laplacian(dim: int, n: int, bc: str):
    """Discrete Laplacian part of S(ξ) and the node weights.

    Returns (Lap, w, e, h):
      Lap  sparse real matrix (T in 1D; D⊗T + T⊗D for absorbing 2D, Theorem A.4;
           I⊗T + T⊗I for Dirichlet 2D, Theorem A.3),
      w    per-node weight of the k² term and of the source (D_2 weights / b_0 weights),
      e    per-node indicator of the absorbing boundary term D_1 (zero for Dirichlet),
      h    mesh size.
    """
    if bc == "absorbing":
        h = 1.0 / (n - 1)
        T = T_absorbing(n, h)
        d = half_weights(n)
        if dim == 1:
            e = np.zeros(n)
            e[0] = e[-1] = 1.0
            return T, d.copy(), e, h
        D = sp.diags(d)
        Lap = (sp.kron(D, T) + sp.kron(T, D)).tocsr()
        w = np.outer(d, d).ravel()          # w[j*n+i] = d_j d_i
        onb = np.zeros(n, dtype=bool)
        onb[0] = onb[-1] = True
        e = (onb[None, :] | onb[:, None]).astype(np.float64).ravel()
        return Lap, w, e, h
    if bc == "dirichlet":
        h = 1.0 / (n + 1)
        T = T_dirichlet(n, h)
        if dim == 1:
            return T, np.ones(n), np.zeros(n), h
        I = sp.identity(n)
        Lap = (sp.kron(I, T) + sp.kron(T, I)).tocsr()
        return Lap, np.ones(n * n), np.zeros(n * n), h
    raise ValueError("bc must be 'absorbing' or 'dirichlet'")


def deterministic_S(dim: int, n: int, bc: str, k: np.ndarray, shift: complex = 1.0) -> sp.csr_matrix:
    """S = Lap - i D_1(k) - shift·D_2(k) for one deterministic wavenumber field k
    (Theorems A.1-A.4; shift = 1+iβ gives the shifted operator of eq. shifted_helmholtz,
    applied to the k² term only, eq. M)."""
    Lap, w, e, h = laplacian(dim, n, bc)
    return (Lap.astype(np.complex128)
            - 1j * sp.diags(e * k / h)
            - shift * sp.diags(w * k * k)).tocsr()
