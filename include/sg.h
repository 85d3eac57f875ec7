/*
 * sg.h - C ABI of the MI355X stochastic-Galerkin Helmholtz solver.
 *
 * Problem (Section 3, eq. stochastic_helmholtz; absorbing BC eq. stochastic_bc_abs):
 *     -Δu - k(x,ξ)² u = f  on (0,1)^d,  ∂_n u - i k u = 0 on the boundary,
 *     k(x,ξ) = k_0(x) + Σ_{ℓ=1..s} ξ_ℓ k_ℓ(x),  ξ_ℓ ~ U[-1,1] independent (Section 2.2).
 * Discretisation: finite differences (Theorems A.2 / A.4) and stochastic Galerkin
 * projection on the orthonormal Legendre chaos of total degree <= r (Section 2.3,
 * Section 3.1).  The result is the complex symmetric system
 *     A V = b,   A = I_{m+1} ⊗ L - i[B_ij] - [C_ij]   (Theorem 3.3, Theorem A.4),
 *     b = [w∘f; 0; ...; 0],
 * with unknown V = [V_0; ...; V_m], m+1 = Q = (s+r)!/(s!r!) (eq. number_basis_polynomial).
 *
 * Vector layout: Q·n^d complex128 values, PC index slowest, then y, then x fastest
 * (eq. LGS_from_FD_G; Theorem A.3 node ordering).  A complex value is two doubles
 * (re, im), the layout of torch.complex128 and hipDoubleComplex.  All vector
 * arguments are DEVICE pointers, 16-byte aligned, owned by the caller; the
 * library never frees them.  Host pointers are marked "host".
 *
 * Errors: a negative return value is a hard failure (outputs undefined); a
 * positive value means the result is valid but see the stats (not converged,
 * fallback used).  No function aborts or throws; sg_last_error() returns a
 * description of the last failure on the calling thread.
 *
 * Threading and streams: one handle serves one stream at a time.  Every call
 * enqueues its work on the given stream; calls that return host results
 * (sg_gmres, sg_fgmres, sg_cgs2, sg_norm, sg_stationary with a history) synchronise
 * that stream.
 */
#ifndef SG_H
#define SG_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } sg_c64;
typedef struct sg_ctx* sg_handle;

enum {
    SG_OK = 0,
    SG_ENOTCONV = 1,        /* maxit reached before tol: x is the last iterate   */
    SG_FALLBACK_USED = 2,   /* learned correction was rejected, plain path used  */
    SG_EINVAL = -1,         /* invalid argument                                   */
    SG_ENOMEM = -2,         /* device or host allocation failed                   */
    SG_EHIP = -3,           /* a HIP runtime call failed                          */
    SG_EBREAKDOWN = -4,     /* Krylov breakdown with a non-solution               */
    SG_ENONFINITE = -5,     /* NaN/Inf met in a residual or Hessenberg entry      */
    SG_ESETUP = -6          /* setup validation failed (eigenfactors, pivots)     */
};

enum { SG_BC_ABSORBING = 0 };

/* Preconditioners (Sections 4-5). */
enum {
    SG_PC_NONE = 0,         /* no preconditioner                                  */
    SG_PC_MEAN = 1,         /* mean value A_0 = I ⊗ S(ξ̄)  (Section 5, eq. bar_A)   */
    SG_PC_CSL_MEAN = 2,     /* mean CSL   M_0 = I ⊗ S_β(ξ̄), k̄² → (1+iβ)k̄² (eq. M) */
    SG_PC_MEAN_NET = 3      /* A_0 followed by the learned correction (sg_net_*)  */
};

/* Arithmetic of the preconditioner's dense transforms; the outer operator,
 * orthogonalisation, least squares and true residual are always FP64. */
enum { SG_PREC_F64 = 0, SG_PREC_F32 = 1, SG_PREC_BF16X3 = 2 };

typedef struct {
    int dim;                  /* 1 or 2                                                     */
    int n;                    /* nodes per side including the boundary (n = q+2 >= 3),
                                 h = 1/(n-1)  (grids grid_1d / grid_2d)                     */
    int bc;                   /* SG_BC_ABSORBING                                            */
    int s;                    /* number of random variables, 1..8                          */
    int degree;               /* total PC degree r, 0..8                                   */
    const double* k_fields;   /* host, (s+1)·n^dim doubles: k_0, ..., k_s at the nodes,
                                 x fastest (eq. random_wavenumber)                          */
    double k_mean;            /* k̄ > 0: the constant mean wavenumber, every entry of k_0 must
                                 equal it; the block solves of A_0 / M_0 use fast
                                 diagonalisation (any precision).  0: k_0 varies in space
                                 (the wedge of Section 7, eq. wavenumber_k123); the block
                                 solves use an exact line-by-line block LU of S(k_0) in
                                 FP64 (2D: n <= 257; its host setup costs O(n^4)).  Any
                                 other value returns SG_EINVAL.                             */
    double csl_beta;          /* β of the CSL shift (Section 4, eq. shifted_helmholtz)      */
} sg_problem;

typedef struct {
    int restart;              /* m of GMRES(m), 1..512                                      */
    int maxit;                /* cap on the total number of inner iterations                */
    int precond;              /* SG_PC_*                                                    */
    int precision;            /* SG_PREC_* for the preconditioner                           */
    double tol;               /* target of the true relative residual ||b-Ax||_2/||b||_2
                                 (left preconditioning: see side)                           */
    int x0_zero;              /* 1: start from x = 0; 0: x holds the initial guess          */
    double* hist;             /* host, optional: residual estimate after each iteration     */
    int hist_cap;             /* capacity of hist                                           */
    int side;                 /* 0: right preconditioning A P^{-1} y = b, x = P^{-1} y (tol
                                 on ||b-Ax||/||b||); 1: left, P^{-1} A x = P^{-1} b (eq.
                                 CSL_preconditioned), whose residual is P^{-1}(b-Ax): tol on
                                 ||P^{-1}(b-Ax)||/||P^{-1}b|| (Section 6.3).  Left is
                                 available in sg_gmres with a built-in preconditioner.      */
} sg_solve_opts;

typedef struct {
    int iters;                /* inner iterations performed                                 */
    int restarts;             /* completed cycles                                           */
    int converged;            /* 1 if the true relative residual <= tol                     */
    int fallback;             /* 1 if the learned correction was switched off               */
    double relres_true;       /* final ||b-Ax||_2/||b||_2 recomputed in FP64                */
    double relres_est;        /* final Arnoldi estimate |g_{j+1}|/||b|| (left: /||P^{-1}b||)  */
    double t_setup;           /* milliseconds                                               */
    double t_precond, t_matvec, t_orth;  /* GPU milliseconds per phase, measured only while
                                 profiling of every kind is on (sg_set_profiling), else 0:
                                 the events between the phases idle the GPU briefly    */
    double t_total;           /* milliseconds                                               */
    double relres_prec;       /* left preconditioning: final ||P^{-1}(b-Ax)||/||P^{-1}b||, the
                                 quantity tol applies to (right: equal to relres_true)      */
} sg_solve_stats;

/* Build the operator for one problem: basis, triple-product tables, coefficient
 * fields, eigenfactors of the 1D mean operator and pivoted tridiagonal factors
 * (host FP64, validated), then upload to the current device.  *out owns all of it.
 * Shapes: every (s, degree) with Q·66·16 + |Γ₂|·512 <= 160 KiB (|Γ₂| = 1+2s+s(s-1)/2, the
 * LDS tile of the generic operator kernel), and beyond that the shapes with a specialised
 * kernel (2D: s = 3 up to degree 8); any other shape returns SG_EINVAL here.
 * The uploads go through a non-blocking stream that the call creates for itself and are
 * complete when it returns (stream is not used), so setups may run in host threads beside
 * solves on other streams without waiting for them. */
int  sg_setup(const sg_problem* prob, hipStream_t stream, sg_handle* out);
void sg_destroy(sg_handle h);

/* Q (number of PC coefficients) and the multi-index table: multi_index may be NULL,
 * else host, Q·s ints, row i = exponents of φ_i (graded order, Section 2.3). */
int  sg_basis(sg_handle h, int* Q, int* multi_index);
/* Unknown count Q·n^dim. */
long long sg_size(sg_handle h);

/* b = [w∘f; 0; ...; 0] with the boundary weights of Theorems A.2 / A.4;
 * f_host: host, n^dim doubles; b_dev: device, Q·n^dim complex. */
int  sg_rhs(sg_handle h, const double* f_host, sg_c64* b_dev, hipStream_t stream);

/* y = A x (Theorem 3.3), FP64, matrix-free; x and y must not overlap. */
int  sg_apply(sg_handle h, const sg_c64* x, sg_c64* y, hipStream_t stream);

/* How the handle solves its mean block (the block solves of A_0 and M_0): SG_MEAN_FD, fast
 * diagonalisation (constant k̄; 1D: the tridiagonal solve); SG_MEAN_LINE, the exact block LU
 * over grid lines (k_mean = 0: spatially varying k_0); SG_MEAN_LINE_FALLBACK, the same block
 * LU chosen at setup because the eigenfactors of a constant-k̄ 2D block failed their checks
 * (residual, D-orthonormality, or cond₂ of the eigenvector matrix Ṽ above 1e4, whose
 * square amplifies the rounding of the transforms); possible for n <= 257, beyond that
 * sg_setup returns SG_ESETUP.  cond_v (may be NULL) receives the figure checked: the bound
 * ||Ṽ||_F ||ṼᵀD||_F, or power-iteration estimates of the two 2-norms when that bound is
 * above 1e3 (2D constant k̄ only, else 0).  The line forms are FP64 only and not served by the batched solver or the
 * learned correction. */
enum { SG_MEAN_FD = 0, SG_MEAN_LINE = 1, SG_MEAN_LINE_FALLBACK = 2 };
int  sg_mean_solver(sg_handle h, int* kind, double* cond_v);
/* Where this handle's sg_setup spent its time, in milliseconds (host array of 4): the whole
 * call, its device allocations, its uploads (copy and wait) and the creation of its upload
 * stream; the rest is host computation. */
int  sg_setup_times(sg_handle h, double* ms);
/* Process-wide limit on that cond₂ figure for later sg_setup calls (default 1e4, >= 1,
 * else SG_EINVAL); a limit of 1 sends every 2D constant-k̄ problem with n <= 257 to the line
 * factorisation. */
int  sg_set_eigen_cond_limit(double limit);

/* Statistics of the SG solution u_m(x,ξ) = Σ_i V_i(x) φ_i(ξ) held in x (Section 7, Figure
 * bE_Var): mean = E[u_m] = V_0 (device, n^dim complex, may be NULL) and var = [Var[Re u_m];
 * Var[Im u_m]] = [Σ_{i>=1} (Re V_i)²; Σ_{i>=1} (Im V_i)²] (device, 2·n^dim doubles, may be
 * NULL, not both).  Asynchronous on the stream. */
int  sg_moments(sg_handle h, const sg_c64* x, sg_c64* mean, double* var, hipStream_t stream);

/* γ_j = max{ ||V_i||_∞ : total degree of φ_i = j } for j = 0..degree (eq. magnitude_V,
 * Figure k123_convergence): gamma_host, host, degree+1 doubles.  Synchronises the stream;
 * SG_ENONFINITE if a coefficient is not finite. */
int  sg_degree_magnitudes(sg_handle h, const sg_c64* x, double* gamma_host, hipStream_t stream);

/* Select the operator of the handle: beta = 0 gives A (the default); beta != 0 gives the
 * full complex shifted Laplace matrix M(beta) = L - iB - (1 + i beta) K = A - i beta K
 * (eq. M, Section 4: only the k² block K is shifted, the boundary block is not).  It applies
 * to sg_apply and to the matrix of sg_gmres, sg_fgmres, sg_stationary and
 * sg_gmres_batched on this handle; the preconditioners and sg_rhs are unchanged.  A second handle of the same problem with
 * beta set solves with the full M, e.g. as the inner solve of a nested FGMRES whose outer
 * matrix is A.  Returns SG_EINVAL for a non-finite beta, or when no operator kernel serves
 * the shifted operator of this shape (shapes with Q > 84 beyond the generic kernel's LDS
 * tile). */
int  sg_set_operator_shift(sg_handle h, double beta);

/* z = P^{-1} r for P = A_0 or M_0 (pc = SG_PC_MEAN / SG_PC_CSL_MEAN) by fast
 * diagonalisation of the mean block (Section 5; Section 6.3 block reuse), in the given
 * precision; SG_PC_NONE copies.  SG_PREC_F32 / SG_PREC_BF16X3 (2D): the transforms in that
 * precision with FP32 accumulation, their intermediate and the tridiagonal sweep in FP32
 * (the factors are FP64 and rounded as they are read); r and z stay FP64.  1D: the sweep is
 * FP64 in every precision.  With a spatially varying mean (k_mean = 0 at setup) the block
 * solve is the line block LU, FP64 only (another precision: SG_EINVAL).  r and z may alias. */
int  sg_precond(sg_handle h, int pc, int precision, const sg_c64* r, sg_c64* z, hipStream_t stream);

/* Restarted GMRES(m), right-preconditioned (eq. preconditioned_2d) or, with opts->side = 1,
 * left-preconditioned (eq. CSL_preconditioned): CGS2 Arnoldi, Givens least squares, true FP64
 * residual (left: preconditioned residual) at each cycle end. */
int  sg_gmres(sg_handle h, const sg_c64* b, sg_c64* x, const sg_solve_opts* opts,
              sg_solve_stats* stats, hipStream_t stream);

/* Orthogonalisation of sg_gmres / sg_fgmres with a built-in preconditioner (restart <= 512):
 * SG_ORTH_DCGS2 (the default), classical Gram-Schmidt with one re-orthogonalisation delayed
 * by one step, so that one pass over the basis re-orthogonalises the previous vector and
 * projects the new one (two passes over the basis per step, one coefficient exchange with
 * the host; the Arnoldi process in the flexible form z_j = P^{-1}u_j, x += Z y);
 * SG_ORTH_CGS2, the same two Gram-Schmidt passes done in the same step (three passes over
 * the basis).  Other solves (callbacks, the learned correction, left preconditioning)
 * always use SG_ORTH_CGS2.  Beyond 64 basis vectors the delayed form reduces over chunks of
 * 64 vectors in one launch and updates chunk by chunk (u and w read and written once more
 * per further chunk).  The delayed form stores each candidate scaled to about unit norm; the
 * two-pass form keeps its basis vectors unnormalised (lazy scales) and stores a vector
 * normalised when its norm leaves [1e-50, 1e50], so that long cycles on a poorly scaled
 * operator (||A P^{-1}|| >> 1, e.g. no preconditioner) do not overflow in either form. */
enum { SG_ORTH_DCGS2 = 0, SG_ORTH_CGS2 = 1 };
int  sg_set_orthogonalisation(sg_handle h, int kind);
/* The orthonormal Arnoldi basis v_0..v_{nvec-1} of the last cycle of the handle's last
 * delayed-CGS2 solve (device, vector-major, owned by the handle, valid until its next solve);
 * for checks of orthogonality. */
int  sg_last_basis(sg_handle h, int* nvec, const sg_c64** V);

/* Flexible GMRES(m): the preconditioner may change between iterations.  cb == NULL
 * uses the built-in opts->precond / opts->precision; otherwise cb(user, r, z, stream)
 * must write z ≈ P^{-1} r (device vectors of sg_size()) and return 0. */
typedef int (*sg_precond_cb)(void* user, const sg_c64* r, sg_c64* z, hipStream_t stream);
int  sg_fgmres(sg_handle h, const sg_c64* b, sg_c64* x, const sg_solve_opts* opts,
               sg_precond_cb cb, void* user, sg_solve_stats* stats, hipStream_t stream);

/* Stationary iteration with the mean-based block matrix B (eq. stationary_iteration,
 * Section 5; B = A_0 for pc = SG_PC_MEAN, M_0 for SG_PC_CSL_MEAN):
 *   x_0 = B^{-1} b,   x_{i+1} = x_i + B^{-1} (b - A x_i),   i = 0 .. iters-1,
 * all in FP64 (no Krylov workspace beyond two scratch vectors).  It converges when the
 * spectral radius of I - B^{-1} A is below one (Theorem 5.3 gives a sufficient bound) and
 * diverges otherwise; the caller judges that from the history.
 * b, x: device vectors of sg_size(), must not overlap; x is overwritten.
 * hist: host, may be NULL, else iters+1 doubles: ||b - A x_i|| / ||b|| for i = 0..iters
 * (each entry costs one stream synchronisation).  A zero b gives x = 0 and a zero
 * history.  Returns SG_ENONFINITE if a history entry is not finite, SG_EINVAL for bad
 * arguments (pc not one of the two, iters < 0). */
int  sg_stationary(sg_handle h, const sg_c64* b, sg_c64* x, int pc, int iters, double* hist,
                   hipStream_t stream);

/* Batched right-preconditioned GMRES(m) over `count` independent problems of any
 * size (instances of a parametric study, each with its own handle).
 * The algorithm per instance is that of sg_gmres (Section 5 preconditioners, Section 6.3
 * block reuse), with the delayed CGS2 in the flexible form (2m+2 vectors of workspace per
 * instance), or with the two-pass CGS2 and x += P^{-1}(V y) (m+3 vectors) when every handle
 * of the batch is set to SG_ORTH_CGS2; the instances advance in lockstep steps, each phase of
 * a step being one grouped kernel launch over all active instances, with one host
 * synchronisation per step.  Instances are admitted from a queue ordered by estimated cost
 * (largest first) into Krylov workspaces carved from one device arena of at most
 * max(largest instance, half the available device memory); the arena is kept for later
 * calls on the same device
 * (allocating it costs more than a batch of solves) until sg_batched_release() or the end of
 * the process, and calls on one device are serialised.
 * handles, b and x: host arrays of `count` entries; b[i], x[i] device vectors of
 * sg_size(handles[i]) complex, x[i] is overwritten (the initial guess is zero, opts
 * x0_zero is ignored).  A handle may appear only once.  opts->restart must be in
 * [1, 63] and opts->side 0; opts->hist is ignored.  stats: host array of `count` entries or NULL
 * (t_precond / t_matvec / t_orth are 0; t_total is the wall time from admission to
 * completion).  The GEMM tile shape of each instance comes from the autotuner table
 * (sg_autotune / sg_tune_set), else a size-based default (3M 32×32 or 64×64 in FP64 and
 * FP32, 64×128 or 64×256 in BF16x3).  Returns SG_OK if every instance
 * converged, SG_ENOTCONV if some did not (their stats say which: converged = 0, a
 * non-finite value gives relres_true = NaN), negative on invalid arguments or a HIP
 * failure.  Kernel timing, when enabled, is recorded in the profiler of handles[0]. */
int  sg_gmres_batched(int count, const sg_handle* handles, const sg_c64* const* b, sg_c64* const* x,
                      const sg_solve_opts* opts, sg_solve_stats* stats, hipStream_t stream);
/* Free the batched solver's arena on the current device (after synchronising the device). */
int  sg_batched_release(void);

/* GEMM tile-shape autotuner of the preconditioner transforms: for every distinct
 * (n, Q) among the 2D handles, times each tile shape (SG_GEMM_TILE_*) available in
 * `precision` on grouped launches of the forward and the inverse transform over up to 8
 * instances of that shape, `reps` repetitions, and stores the fastest in a process-wide
 * table keyed by (n, Q, precision).  Uses the handles' preconditioner scratch (their
 * contents are overwritten) and a temporary device buffer.  *ms_total (may be NULL)
 * receives the measured GPU time. */
/* Expanded real form (BM x BN real columns; the 256-wide tiles FP32 / BF16x3 only), and
 * the 3M complex form (FP64 and FP32; BM x BN complex columns, three real products per
 * complex multiply-add). */
enum { SG_GEMM_TILE_128x128 = 0, SG_GEMM_TILE_64x128 = 1, SG_GEMM_TILE_64x64 = 2, SG_GEMM_TILE_64x32 = 3,
       SG_GEMM_TILE_32x64 = 4, SG_GEMM_TILE_3M_32x32 = 5, SG_GEMM_TILE_3M_64x32 = 6, SG_GEMM_TILE_3M_32x64 = 7,
       SG_GEMM_TILE_3M_64x64 = 8, SG_GEMM_TILE_64x256 = 9, SG_GEMM_TILE_128x256 = 10 };
int  sg_autotune(int count, const sg_handle* handles, int precision, int reps, double* ms_total,
                 hipStream_t stream);
/* Read (-1 if absent) or set one entry of the autotuner table; sg_tune_set returns
 * SG_EINVAL for a shape not available in that precision (3M shapes: FP64 and FP32; 64x256
 * and 128x256: FP32 and BF16x3 only). */
int  sg_tune_get(int n, int Q, int precision);
int  sg_tune_set(int n, int Q, int precision, int tile);

/* One CGS2 step: orthogonalise w (n complex) against the nv orthonormal columns of
 * V (nv·n complex, vector-major) twice, normalise it in place, and return the nv+1
 * Arnoldi coefficients h_host[0..nv-1] = V^H w (both passes summed), h_host[nv] = ||w||. */
int  sg_cgs2(long long n, int nv, const sg_c64* V, sg_c64* w, sg_c64* h_host, hipStream_t stream);

/* sg_cgs2 for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same kernels and the same
 * results, bit for bit, but the reduction partials and coefficients live in a fixed
 * file-scope device array of 2 MiB + 3 KiB per GPU (held until the process ends) instead of
 * buffers allocated per call, and the coefficients go to the host through h_host itself.
 * Limit: nv <= 64 (SG_EINVAL above it).  Calls no hipMalloc / hipFree / hipHostMalloc.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (two
 * streams, two threads) race and must be serialised by the caller.  Synchronises the
 * stream. */
int  sg_cgs2_noalloc(long long n, int nv, const sg_c64* V, sg_c64* w, sg_c64* h_host, hipStream_t stream);

/* ||x||_2 in FP64 (deterministic two-stage reduction). */
int  sg_norm(long long n, const sg_c64* x, double* out_host, hipStream_t stream);

/* out = alpha x + beta y over n complex entries (device vectors; out may alias x or y; y may
 * be NULL when beta = 0): the vector update of the solvers (the residual b - A x and the
 * iterate update, Section 6.3), exposed for callers that form residuals and errors on the
 * device, e.g. the learned form's training pairs.  Asynchronous on the stream. */
int  sg_axpby(long long n, sg_c64 alpha, const sg_c64* x, sg_c64 beta, const sg_c64* y, sg_c64* out,
              hipStream_t stream);

/* Per-kernel-class timing with HIP events recorded on the launch stream around every
 * kernel the handle issues (off by default).  Classes: */
enum {
    SG_K_APPLY = 0,     /* SG operator                 (algorithmic bytes)            */
    SG_K_GEMM = 1,      /* preconditioner transforms   (algorithmic flops)            */
    SG_K_TRI = 2,       /* tridiagonal sweeps          (algorithmic bytes)            */
    SG_K_DOT = 3,       /* CGS2 multi-dot              (algorithmic bytes)            */
    SG_K_AXPY = 4,      /* CGS2 multi-axpy / updates   (algorithmic bytes)            */
    SG_K_NORM = 5,      /* norms and second-stage reductions (algorithmic bytes)      */
    SG_K_NET = 6,       /* correction network convolutions (algorithmic flops)        */
    SG_K_NKINDS = 8
};
/* on != 0 enables recording (of every kind) and clears the counters. */
int  sg_set_profiling(sg_handle h, int on);
/* Restrict recording to the kinds whose bit (1u << kind) is set in mask (after
 * sg_set_profiling, which resets the mask to all kinds). */
int  sg_profile_kinds(sg_handle h, unsigned mask);
/* Synchronises the pending events and returns, per class k < nkinds (host arrays of
 * nkinds entries, any may be NULL): total milliseconds, launch count, and the summed
 * algorithmic work (bytes or flops as listed above). */
int  sg_kernel_times(sg_handle h, int nkinds, double* ms, long long* count, double* work);

/* ---- Learned correction network ----------------------------------------------------
 * A 3-level convolutional U-Net (widths 32, 64, 128; 3×3 convolutions with ReLU, 2×2
 * average pooling, nearest upsampling with skip concatenation, linear 1×1 head) that
 * maps a residual v (2Q channels: Re, Im of each PC block, scaled to unit RMS) and the
 * s+1 wavenumber coefficient fields k_l/k̄ to a correction of the mean-value block solve
 * A_0^{-1} v (Section 5), used as the preconditioner
 *     z = A_0^{-1} v + ||A_0^{-1} v|| / sqrt(Q n²) · N(v)
 * inside flexible GMRES (pc = SG_PC_MEAN_NET).  Tensors are BF16 with FP32 accumulation on
 * the matrix cores; master weights, gradients and Adam state are FP32.  Parameters are a
 * flat FP32 vector: per layer W[c_out][k][k][c_in] then b[c_out], layers enc0a, enc0b,
 * enc1a, enc1b, bota, botb, dec1a, dec1b, dec0a, dec0b, head. */
typedef struct sg_net_s* sg_net;
/* Network for Q PC coefficients and s random variables (c_in = 2Q+s+1, c_out = 2Q),
 * He-normal weights from a SplitMix64 stream seeded by `seed`; on the current device. */
int  sg_net_create(int Q, int s, unsigned long long seed, sg_net* out);
void sg_net_destroy(sg_net net);
long long sg_net_num_params(sg_net net);
/* Host FP32 arrays of sg_net_num_params entries; set also resets the Adam state. */
int  sg_net_get_params(sg_net net, float* host);
int  sg_net_set_params(sg_net net, const float* host);
/* Forward pass on `batch` NHWC images of H×H pixels (H a multiple of 4): x device FP32
 * [batch][H][H][c_in], y device FP32 [batch][H][H][c_out]. */
int  sg_net_forward_nhwc(sg_net net, int batch, int H, const float* x, float* y, hipStream_t stream);
/* Mean squared error against t (device FP32 [batch][H][H][c_out]) and its gradient with
 * respect to the parameters (kept for sg_net_adam_step; copied to grad_host if not NULL). */
int  sg_net_grad_nhwc(sg_net net, int batch, int H, const float* x, const float* t, double* loss,
                      float* grad_host, hipStream_t stream);
/* One Adam step (β1 0.9, β2 0.999, ε 1e-8) with the last computed gradient. */
int  sg_net_adam_step(sg_net net, float lr, hipStream_t stream);
/* One training step on `batch` pairs (r_i, e_i) with A e_i = r_i of the problems
 * handles[i] (2D, same n, Q and s as the network): target N(r_i) = e_i - A_0^{-1} r_i in
 * the units above, A_0^{-1} in `precision`; mean loss returned in *loss (may be NULL). */
int  sg_net_train_pairs(sg_net net, int batch, const sg_handle* handles, const sg_c64* const* r,
                        const sg_c64* const* e, float lr, int precision, double* loss, hipStream_t stream);
/* Binary parameter file (header with Q, s and the parameter count, then FP32 values). */
int  sg_net_save(sg_net net, const char* path);
int  sg_net_load(sg_net net, const char* path);
/* Attach a network (not owned; NULL detaches) to a handle for SG_PC_MEAN_NET.  With it,
 * sg_precond computes the learned preconditioner (r and z must not alias) and sg_fgmres
 * runs one cycle of flexible GMRES with it; if that cycle does not reach the tolerance
 * (or the network yields non-finite values), plain A_0-preconditioned GMRES continues
 * from the current iterate (from zero if it is not finite) and the call returns
 * SG_FALLBACK_USED with stats->fallback = 1. */
int  sg_attach_net(sg_handle h, sg_net net);

const char* sg_strerror(int status);
const char* sg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SG_H */
