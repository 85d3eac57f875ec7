"""Preconditioners by sparse LU, as the paper implements them (Section 6.3).

* Mean value preconditioner A_0 = I_{m+1} ⊗ S(ξ̄) (Section 5, eq. bar_A): one LU
  of the n×n block S(ξ̄) is reused for all m+1 blocks by reshaping the vector
  to an n×(m+1) array and solving the m+1 right-hand sides together.
* Mean CSL preconditioner M_0 = I_{m+1} ⊗ (S(ξ̄) with k̄² → (1+iβ)k̄²)
  (Sections 4 and 6): the same block solve with the shifted block.
* Full CSL preconditioner M(β) = A - iβK (eq. M): one LU of the whole system.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .assemble import SGSystem, mean_block


class BlockLU:
    """z = (I_Q ⊗ S)^{-1} v with one sparse LU of S (Section 6.3 reshape trick)."""

    def __init__(self, S, Q: int):
        self.lu = spla.splu(S.tocsc())
        self.Q = Q
        self.P = S.shape[0]

    def __call__(self, v: np.ndarray) -> np.ndarray:
        V = np.asarray(v, dtype=np.complex128).reshape(self.Q, self.P)
        return self.lu.solve(np.ascontiguousarray(V.T)).T.reshape(-1)


class FullLU:
    def __init__(self, M):
        self.lu = spla.splu(M.tocsc())

    def __call__(self, v: np.ndarray) -> np.ndarray:
        return self.lu.solve(np.asarray(v, dtype=np.complex128))


def mean_value(sys_: SGSystem) -> BlockLU:
    """A_0^{-1}: the mean value preconditioner (Section 5)."""
    return BlockLU(mean_block(sys_, 1.0), sys_.Q)


def mean_csl(sys_: SGSystem, beta: float) -> BlockLU:
    """M_0^{-1}: mean value CSL preconditioner (shift on the k² term only, eq. M)."""
    return BlockLU(mean_block(sys_, 1.0 + 1j * beta), sys_.Q)


def full_csl(sys_: SGSystem, beta: float) -> FullLU:
    """M(β)^{-1} for the full CSL preconditioner (eq. M)."""
    return FullLU(sys_.csl(beta))


def direct_solve(sys_: SGSystem, b: np.ndarray | None = None) -> np.ndarray:
    """x = A \\ b by sparse LU (SuperLU; the paper uses UMFPACK)."""
    rhs = sys_.b if b is None else b
    return spla.splu(sys_.A.tocsc()).solve(np.asarray(rhs, dtype=np.complex128))
