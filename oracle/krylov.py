"""Textbook Krylov solvers (Saad-Schultz GMRES; Section 6.3 and Section 7 usage).

gmres   restarted GMRES(m) with *right* preconditioning: solves A M^{-1} y = b,
        x = M^{-1} y (eq. CSL_preconditioned, eq. preconditioned_2d).  Modified
        Gram-Schmidt Arnoldi and complex Givens rotations.  The stopping test is
        the relative residual of the unpreconditioned system ||b - Ax||/||b||
        (Section 6.3): during a cycle its Arnoldi estimate |g_{j+1}|/||b|| is used,
        and at the end of each cycle the true residual is recomputed; a cycle
        whose true relative residual is above tol is followed by a restart.
        restart >= maxit gives full GMRES (no restarts) as used in the paper.
gmres_left  restarted GMRES(m) with *left* preconditioning, M^{-1} A x = M^{-1} b (eq.
        CSL_preconditioned); residual and stopping test on M^{-1} r (Section 6.3).
fgmres  flexible variant that stores the preconditioned vectors Z (Saad 1993).
stationary  the iteration B x^{(i+1)} = b - (A - B) x^{(i)} with B = A_0 and
        x^{(0)} = A_0^{-1} b (eq. stationary_iteration, eq. stationary_iteration_A0).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class SolveInfo:
    iters: int = 0
    cycles: int = 0
    converged: bool = False
    relres_true: float = np.inf
    breakdown: bool = False
    hist: list = field(default_factory=list)
    relres_prec: float = np.inf   # left preconditioning: ||M^{-1}(b - Ax)|| / ||M^{-1}b||
    H: np.ndarray | None = None   # Hessenberg of the last cycle (unrotated)
    V: np.ndarray | None = None   # Arnoldi basis of the last cycle


def givens(a: complex, b: complex):
    """(c, s) with c real such that [[c, s], [-conj(s), c]] @ [a, b] = [r, 0]."""
    if b == 0:
        return 1.0, 0.0
    if a == 0:
        return 0.0, 1.0 * np.conj(b) / abs(b)
    t = np.hypot(abs(a), abs(b))
    c = abs(a) / t
    s = (a / abs(a)) * np.conj(b) / t
    return c, s


def _identity(v):
    return v


def gmres(A, b, M=None, restart: int = 50, tol: float = 1e-8, maxit: int = 10000,
          x0=None, flexible: bool = False, keep_basis: bool = False):
    """Right-preconditioned restarted GMRES(m) / FGMRES(m).

    A, M are callables v -> A v and v -> M^{-1} v.  Returns (x, SolveInfo).
    """
    M = M or _identity
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    info = SolveInfo()
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    if bnorm == 0.0:
        info.converged, info.relres_true = True, 0.0
        return np.zeros_like(b), info
    m = int(max(1, min(restart, maxit, b.size)))
    while True:
        r = b - A(x)
        beta = np.linalg.norm(r)
        info.relres_true = beta / bnorm
        if info.relres_true <= tol:
            info.converged = True
            break
        if info.iters >= maxit:
            break
        info.cycles += 1
        V = np.zeros((m + 1, b.size), dtype=np.complex128)
        Z = np.zeros((m, b.size), dtype=np.complex128) if flexible else None
        H = np.zeros((m + 1, m), dtype=np.complex128)
        R = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            z = M(V[j])
            if flexible:
                Z[j] = z
            w = A(z)
            for i in range(j + 1):                 # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            col = H[: j + 2, j].copy()
            for i in range(j):                     # previous rotations
                t = cs[i] * col[i] + sn[i] * col[i + 1]
                col[i + 1] = -np.conj(sn[i]) * col[i] + cs[i] * col[i + 1]
                col[i] = t
            cs[j], sn[j] = givens(col[j], col[j + 1])
            col[j] = cs[j] * col[j] + sn[j] * col[j + 1]
            col[j + 1] = 0.0
            R[: j + 2, j] = col
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            info.iters += 1
            k = j + 1
            est = abs(g[j + 1]) / bnorm
            info.hist.append(est)
            hnorm = np.linalg.norm(H[: j + 2, j])
            if H[j + 1, j].real <= 1e-14 * max(hnorm, 1e-300):
                info.breakdown = True
                break
            V[j + 1] = w / H[j + 1, j]
            if est <= tol or info.iters >= maxit:
                break
        y = np.linalg.solve(np.triu(R[:k, :k]), g[:k]) if k > 0 else np.zeros(0)
        if flexible:
            x = x + Z[:k].T @ y
        else:
            x = x + M(V[:k].T @ y)
        if keep_basis:
            info.H, info.V = H[: k + 1, :k], V[: k + 1]
        if info.breakdown:
            r = b - A(x)
            info.relres_true = np.linalg.norm(r) / bnorm
            info.converged = info.relres_true <= tol
            break
    return x, info


def gmres_left(A, b, M=None, restart: int = 50, tol: float = 1e-8, maxit: int = 10000, x0=None):
    """Left-preconditioned restarted GMRES(m): Arnoldi on M^{-1}A with the start vector
    M^{-1}(b - A x) (the second system of eq. CSL_preconditioned).  Its residual is the
    preconditioned one, M^{-1} r (Section 6.3), so the stopping test is
    ||M^{-1}(b - A x)|| / ||M^{-1} b|| <= tol: the Arnoldi estimate |g_{j+1}| / ||M^{-1} b||
    during a cycle, the recomputed value at each cycle end.  The update is x += V y (no
    preconditioner application).  Modified Gram-Schmidt and complex Givens rotations as in
    ``gmres``.  ``info.relres_prec`` holds the final preconditioned relative residual and
    ``info.relres_true`` the unpreconditioned ||b - Ax|| / ||b||."""
    M = M or _identity
    b = np.asarray(b, dtype=np.complex128)
    info = SolveInfo()
    bp = M(b)
    bpnorm = np.linalg.norm(bp)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    if bnorm == 0.0:
        info.converged, info.relres_true, info.relres_prec = True, 0.0, 0.0
        return np.zeros_like(b), info
    m = int(max(1, min(restart, maxit, b.size)))
    while True:
        r = M(b - A(x))
        beta = np.linalg.norm(r)
        info.relres_prec = beta / bpnorm
        if info.relres_prec <= tol:
            info.converged = True
            break
        if info.iters >= maxit:
            break
        info.cycles += 1
        V = np.zeros((m + 1, b.size), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        R = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            w = M(A(V[j]))
            for i in range(j + 1):                 # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            col = H[: j + 2, j].copy()
            for i in range(j):
                t = cs[i] * col[i] + sn[i] * col[i + 1]
                col[i + 1] = -np.conj(sn[i]) * col[i] + cs[i] * col[i + 1]
                col[i] = t
            cs[j], sn[j] = givens(col[j], col[j + 1])
            col[j] = cs[j] * col[j] + sn[j] * col[j + 1]
            col[j + 1] = 0.0
            R[: j + 2, j] = col
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            info.iters += 1
            k = j + 1
            est = abs(g[j + 1]) / bpnorm
            info.hist.append(est)
            hnorm = np.linalg.norm(H[: j + 2, j])
            if H[j + 1, j].real <= 1e-14 * max(hnorm, 1e-300):
                info.breakdown = True
                break
            V[j + 1] = w / H[j + 1, j]
            if est <= tol or info.iters >= maxit:
                break
        y = np.linalg.solve(np.triu(R[:k, :k]), g[:k]) if k > 0 else np.zeros(0)
        x = x + V[:k].T @ y
        if info.breakdown:
            info.relres_prec = np.linalg.norm(M(b - A(x))) / bpnorm
            info.converged = info.relres_prec <= tol
            break
    info.relres_true = np.linalg.norm(b - A(x)) / bnorm
    return x, info


def fgmres(A, b, M=None, **kw):
    """Flexible GMRES(m): x += Z y with Z = [M_0^{-1}v_0, ...] stored."""
    return gmres(A, b, M, flexible=True, **kw)


def stationary(A, b, Binv, iters: int, x_ref=None):
    """Stationary iteration with B = A_0 started at x0 = A_0^{-1} b
    (eq. stationary_iteration_A0).  Returns (x, errors) with max-norm relative
    errors against x_ref when given."""
    x = Binv(b)
    errs = []
    for _ in range(iters):
        if x_ref is not None:
            errs.append(np.max(np.abs(x - x_ref)) / np.max(np.abs(x_ref)))
        x = x + Binv(b - A(x))
    if x_ref is not None:
        errs.append(np.max(np.abs(x - x_ref)) / np.max(np.abs(x_ref)))
    return x, errs
