"""Assembly of the stochastic Galerkin system A V = b (Theorem 3.3, Theorems A.1-A.4).

    A = I_{m+1} ⊗ L  -  i [B_ij]  -  [C_ij],
    B_ij = diag( e ∘ b_ij(x) / h ),   C_ij = diag( w ∘ c_ij(x) ),
    b    = [ w ∘ f ; 0 ; ... ; 0 ],

with b_ij(x) = ⟨k(x,ξ)φ_i, φ_j⟩ and c_ij(x) = ⟨k(x,ξ)²φ_i, φ_j⟩ (eqs. b_ij, c_ij),
e the absorbing-boundary indicator and w the half/quarter boundary weights of
Theorems A.2 / A.4.  The block index (PC index) is slow, the node index fast
(eq. LGS_from_FD_G, Section A.4 ordering).  For the CSL operator
M(β) = A - iβK (eq. M) the k² part K = [C_ij] is kept separately.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import fd, pc


@dataclass
class SGSystem:
    dim: int
    n: int
    bc: str
    s: int
    degree: int
    Q: int
    P: int
    h: float
    alpha: np.ndarray          # (Q, s) multi-indices
    E: np.ndarray              # (s+1, s+1, Q, Q) moment tables
    Lap: sp.csr_matrix         # I_Q ⊗ L
    Bnd: sp.csr_matrix         # [B_ij]   (real)
    K: sp.csr_matrix           # [C_ij]   (real, SPD)
    A: sp.csr_matrix           # Lap - i Bnd - K
    b: np.ndarray              # right-hand side
    w: np.ndarray
    e: np.ndarray
    k_fields: np.ndarray

    def csl(self, beta: float) -> sp.csr_matrix:
        """M(β) = L - iB - (1+iβ)K = A - iβK (eq. M)."""
        return (self.A - 1j * beta * self.K).tocsr()

    def matvec(self, v: np.ndarray) -> np.ndarray:
        return self.A @ v


def _kron_sum(terms, Q: int, P: int) -> sp.csr_matrix:
    acc = sp.csr_matrix((Q * P, Q * P))
    for table, field in terms:
        if not np.any(table) or not np.any(field):
            continue
        acc = acc + sp.kron(sp.csr_matrix(table), sp.diags(field), format="csr")
    return acc.tocsr()


def sg_system(dim: int, n: int, bc: str, k_fields: np.ndarray, degree: int,
              f: np.ndarray | None = None) -> SGSystem:
    """Assemble A (and b if f is given) for one problem instance."""
    k_fields = np.asarray(k_fields, dtype=np.float64)
    s = k_fields.shape[0] - 1
    Lap1, w, e, h = fd.laplacian(dim, n, bc)
    P = Lap1.shape[0]
    if k_fields.shape[1] != P:
        raise ValueError("k_fields must have n**dim columns")
    alpha = pc.multi_indices(s, degree)
    Q = alpha.shape[0]
    E = pc.moment_tables(s, degree)
    Bterms, Cterms = pc.k_coupling(k_fields, E)
    Lap = sp.kron(sp.identity(Q), Lap1, format="csr")
    Bnd = _kron_sum([(t, e * fld / h) for t, fld in Bterms], Q, P)
    K = _kron_sum([(t, w * fld) for t, fld in Cterms], Q, P)
    A = (Lap.astype(np.complex128) - 1j * Bnd - K).tocsr()
    A.eliminate_zeros()
    b = np.zeros(Q * P, dtype=np.complex128)
    if f is not None:
        b[:P] = w * np.asarray(f, dtype=np.float64)
    return SGSystem(dim, n, bc, s, degree, Q, P, h, alpha, E, Lap, Bnd, K, A, b, w, e, k_fields)


def from_instance(inst) -> SGSystem:
    """Assemble the system for a ``workloads.Instance``."""
    return sg_system(inst.dim, inst.n, inst.bc, inst.k_fields, inst.degree, inst.f)


def mean_block(sys_: SGSystem, shift: complex = 1.0) -> sp.csr_matrix:
    """S(ξ̄) at the mean ξ̄ = E[ξ] = 0, i.e. the deterministic operator with k = k_0
    (Section 5, eq. bar_A); shift = 1+iβ gives the mean CSL block of M_0 (Section 6)."""
    return fd.deterministic_S(sys_.dim, sys_.n, sys_.bc, sys_.k_fields[0], shift)


def apply_at_points(inst, x: np.ndarray, points) -> np.ndarray:
    """(A x) at the rows of the given grid points, for every block i, evaluated point by
    point from Theorem A.4 / A.2 and eqs. b_ij, c_ij without assembling A:

        (A x)_i(p) = (L x_i)(p) - w_p Σ_j c_ij(p) x_j(p) - i (e_p/h) Σ_j b_ij(p) x_j(p).

    Returns an array of shape (Q, len(points)).  Used for sampled checks at sizes where the
    assembled matrix would not fit.
    """
    points = np.asarray(points, dtype=np.int64)
    Lap1, w, e, h = fd.laplacian(inst.dim, inst.n, inst.bc)
    E = pc.moment_tables(inst.s, inst.degree)
    Q = E.shape[2]
    P = Lap1.shape[0]
    X = np.asarray(x, dtype=np.complex128).reshape(Q, P)
    LX = np.asarray((Lap1.tocsr()[points] @ X.T).T)
    kf = np.asarray(inst.k_fields, dtype=np.float64)
    out = np.empty((Q, points.size), dtype=np.complex128)
    for t, p in enumerate(points):
        kp = kf[:, p]
        Cp = np.einsum("a,b,abij->ij", kp, kp, E)
        Bp = np.einsum("a,aij->ij", kp, E[:, 0])
        out[:, t] = LX[:, t] - w[p] * (Cp @ X[:, p]) - 1j * (e[p] / h) * (Bp @ X[:, p])
    return out
