"""CPU FP64 oracle for the stochastic-Galerkin finite-difference Helmholtz system.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  It
is a plain, slow, obviously-correct restatement of the paper (Pulch & Sète,
"The Helmholtz equation with uncertainties in the wavenumber"): it assembles
the sparse SG matrix from the paper's formulas (Theorems A.1-A.4, Lemma 3.1,
eqs. c_ij / b_ij) and solves it by sparse direct factorisation and by textbook
GMRES with sparse-LU block preconditioners (Sections 4-7).  It shares no code,
table or constant with the GPU path; it never imports the GPU package.

Modules
  pc        orthonormal Legendre chaos basis and moment tables E[ξ_a ξ_b φ_i φ_j]
  fd        finite-difference building blocks T, L, boundary weights (Appendix A)
  assemble  the SG matrix A = I⊗L - i[B_ij] - [C_ij] and right-hand side
  precond   mean-value (A_0), mean-CSL (M_0) and full CSL (M) preconditioners via sparse LU
  krylov    restarted right-preconditioned GMRES(m), FGMRES(m), stationary iteration
  spectral  dense condition numbers, spectra and norm bounds (Theorems 4.1, 5.1, 5.3)
  moments   E[u], Var[Re u], Var[Im u] of the SG solution by quadrature over ξ, and the
            per-degree magnitudes of eq. magnitude_V (Section 7)
  unet      numpy reference of the convolutional correction network of the learned
            preconditioner (forward, backward, Adam, SG vector <-> tensor maps)

Parity status: every function is pinned by tests against values printed in
the paper, closed forms or invariants.  ``unet`` has no counterpart in the paper
(parity unpinned against the paper); it is pinned against library correlation,
adjoint identities, central finite differences and the closed-form Adam step.
"""
