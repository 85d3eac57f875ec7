"""Dense spectral tools for small systems (Sections 4-6).

cond2            2-norm condition number (Section 6.2, Figure cond_A).
eig_pencil       spectrum of A M^{-1} (= spectrum of the pencil (A, M); Theorem 4.1 step 1).
disk_margin      how far eigenvalues lie outside the disk |z - 1/2| <= 1/2 (Theorem 4.1).
frobenius_bound  both sides of Theorem 5.1.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def dense(M) -> np.ndarray:
    return M.toarray() if hasattr(M, "toarray") else np.asarray(M)


def cond2(M) -> float:
    sv = np.linalg.svd(dense(M), compute_uv=False)
    return float(sv[0] / sv[-1])


def cond2_right_prec(A, M) -> float:
    """κ_2(A M^{-1})."""
    Ad, Md = dense(A), dense(M)
    return cond2(np.linalg.solve(Md.T, Ad.T).T)


def eig_pencil(A, M) -> np.ndarray:
    """Eigenvalues σ of A x = σ M x, i.e. of M^{-1}A and of A M^{-1}."""
    return sla.eigvals(dense(A), dense(M))


def disk_excess(sig: np.ndarray) -> float:
    """max(|σ - 1/2| - 1/2): <= 0 when every σ lies in the disk of eq. inclusion_disk."""
    return float(np.max(np.abs(sig - 0.5) - 0.5))


def phi_product_norms(s: int, r: int) -> float:
    """Σ_{i,j} ||φ_i φ_j||²_{L²} from the univariate fourth moments (Theorem 5.1, C_m)."""
    from .pc import multi_indices, orthonormal_legendre
    alpha = multi_indices(s, r)
    nodes, weights = np.polynomial.legendre.leggauss(2 * r + 2)
    weights = weights / 2.0
    phi = orthonormal_legendre(r, nodes)
    # F[a,b] = E[φ_a² φ_b²] in one variable
    F = (phi ** 2 * weights) @ (phi ** 2).T
    total = 0.0
    for i in range(alpha.shape[0]):
        for j in range(alpha.shape[0]):
            v = 1.0
            for l in range(s):
                v *= F[alpha[i, l], alpha[j, l]]
            total += v
    return total


def frobenius_bound(sys_, S_mean, DeltaS_L2F: float):
    """Return (lhs, rhs) of Theorem 5.1:
    ||Ā^{-1}A - I||_F <= C_m ||S(ξ̄)^{-1}||_F || ||ΔS(ξ)||_F ||_{L²}."""
    Q = sys_.Q
    Ad = dense(sys_.A)
    Sinv = np.linalg.inv(dense(S_mean))
    Abar_inv = np.kron(np.eye(Q), Sinv)
    lhs = np.linalg.norm(Abar_inv @ Ad - np.eye(Ad.shape[0]), "fro")
    Cm = np.sqrt(Q) * np.sqrt(phi_product_norms(sys_.s, sys_.degree))
    rhs = Cm * np.linalg.norm(Sinv, "fro") * DeltaS_L2F
    return float(lhs), float(rhs)
