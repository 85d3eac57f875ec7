// Restarted GMRES(m) with right preconditioning and delayed CGS2 orthogonalisation, the
// driver of sg_gmres / sg_fgmres for the built-in preconditioners.
//
// The Arnoldi process is written in the flexible form: z_j = P^{-1} u_j is kept (Z basis),
// w_j = A z_j, and A Z_k = V_{k+1} H_k holds for whatever z_j the preconditioner returned,
// so the same driver serves the FP64 preconditioner (where it generates the same Krylov
// space as right-preconditioned GMRES, eq. preconditioned_2d) and the reduced-precision ones
// (flexible GMRES).  The update is x += Z y with y minimising ||β e_1 - H y|| (Givens
// rotations), and at each cycle end the true FP64 residual ||b - Ax||/||b|| decides between
// stopping and restarting (Section 6.3).
//
// Orthogonalisation: classical Gram-Schmidt with one re-orthogonalisation, the second pass
// delayed by one step so that one pass over the basis computes both the re-orthogonalisation
// of the previous candidate u_j and the projection of the new vector w_j (kernels in
// krylov.hip; delayed CGS2 after Hernández, Román & Tomás 2007 and Świrydowicz et al. 2021).
// Column j-1 of H is therefore complete one step later, at step j.  Near convergence the
// host predicts the next column from the Pythagorean norm ||u_{j+1}||² = ||w_j||² - ||h||²;
// when the prediction reaches the tolerance (or the cycle is full) the next step is only a
// finishing reduction of u_{j+1}, without a preconditioner or operator application.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "sg_internal.h"

namespace sgi {

namespace {

struct Timer {
    hipEvent_t e[4] = {};
    bool ok = false;
    explicit Timer(bool on) {
        if (!on) return;
        ok = true;
        for (auto& x : e) ok = ok && hipEventCreateWithFlags(&x, hipEventDisableSystemFence) == hipSuccess;
    }
    ~Timer() {
        for (auto& x : e)
            if (x) (void)hipEventDestroy(x);
    }
    void record(int i, hipStream_t st) {
        if (ok && hipEventRecord(e[i], st) != hipSuccess) ok = false;
    }
    float between(int a, int b) {
        float ms = 0;
        if (ok && hipEventSynchronize(e[b]) == hipSuccess && hipEventElapsedTime(&ms, e[a], e[b]) == hipSuccess)
            return ms;
        return 0.f;
    }
};

int poll(hipEvent_t ev) {
    hipError_t e;
    while ((e = hipEventQuery(ev)) == hipErrorNotReady) {
    }
    SG_HIP(e);
    return SG_OK;
}

using cd = std::complex<double>;

// Givens state of one cycle (complex rotations with real cosines, as in the oracle).
struct Givens {
    int m;
    std::vector<cd> R, g, sn;
    std::vector<double> cs;
    explicit Givens(int m_) : m(m_), R((size_t)(m_ + 1) * m_), g(m_ + 1), sn(m_), cs(m_) {}
    // rotate column j (entries col[0..j+1]); returns |g_{j+1}| after the new rotation. With
    // commit = false nothing is stored (a prediction).
    double add(int j, std::vector<cd> col, bool commit) {
        for (int i = 0; i < j; ++i) {
            const cd t = cs[i] * col[i] + sn[i] * col[i + 1];
            col[i + 1] = -std::conj(sn[i]) * col[i] + cs[i] * col[i + 1];
            col[i] = t;
        }
        const cd a = col[j], bb = col[j + 1];
        double cj;
        cd sj;
        if (std::abs(bb) == 0.0) { cj = 1.0; sj = 0.0; }
        else if (std::abs(a) == 0.0) { cj = 0.0; sj = std::conj(bb) / std::abs(bb); }
        else {
            const double t = std::hypot(std::abs(a), std::abs(bb));
            cj = std::abs(a) / t;
            sj = (a / std::abs(a)) * std::conj(bb) / t;
        }
        const cd gnext = -std::conj(sj) * g[j];
        if (commit) {
            cs[j] = cj;
            sn[j] = sj;
            col[j] = cj * a + sj * bb;
            col[j + 1] = 0.0;
            for (int i = 0; i <= j + 1; ++i) R[(size_t)i * m + j] = col[i];
            g[j + 1] = gnext;
            g[j] = cj * g[j];
        }
        return std::abs(gnext);
    }
};

}  // namespace

// Extra buffers of the delayed CGS2 driver inside the handle's workspace.
static int ensure_dcgs(Ctx* c, int m) {
    Workspace& w = c->ws;
    if (w.dpart && w.dsmall && w.hrec && w.dm >= m) return SG_OK;
    (void)hipFree(w.dpart);
    (void)hipFree(w.dsmall);
    if (w.hrec) (void)hipHostFree(w.hrec);
    w.dpart = w.dsmall = w.hrec = w.hrec_dev = nullptr;
    w.dm = 0;
    if (device_alloc((void**)&w.dpart, (size_t)w.npartial_blocks * (2 * m + 3) * sizeof(double2)) != hipSuccess ||
        device_alloc((void**)&w.dsmall, (size_t)(10 * m + 16) * sizeof(double2)) != hipSuccess)
        return fail(SG_ENOMEM, "delayed CGS2 buffer allocation failed");
    // coherent: the coefficient kernel's stores to the records reach host memory directly
    // (no copy launch per Arnoldi step); the host reads a record after the step's event
    SG_HIP(hipHostMalloc(&w.hrec, (size_t)2 * (2 * m + 3) * sizeof(double2), hipHostMallocCoherent));
    SG_HIP(hipHostGetDevicePointer((void**)&w.hrec_dev, w.hrec, 0));
    w.dm = m;
    return SG_OK;
}

bool dcgs2_serves(const Ctx*, const sg_solve_opts* o, sg_precond_cb cb) {
    return o && !cb && o->side == 0 && o->restart >= 1 && o->restart <= 512 &&
           (o->precond == SG_PC_NONE || o->precond == SG_PC_MEAN || o->precond == SG_PC_CSL_MEAN);
}

int run_gmres_dcgs2(Ctx* c, const double2* b, double2* x, const sg_solve_opts* o, sg_solve_stats* st,
                    hipStream_t stream) {
    auto t_start = std::chrono::steady_clock::now();
    if (!o || !b || !x) return fail(SG_EINVAL, "null argument");
    if (o->maxit < 1) return fail(SG_EINVAL, "maxit must be >= 1");
    if (!(o->tol > 0)) return fail(SG_EINVAL, "tol must be positive");
    const int m = o->restart;
    int rc = ensure_workspace(c, m, true);
    if (rc) return rc;
    if ((rc = ensure_dcgs(c, m))) return rc;
    Workspace& W = c->ws;
    const long long n = c->nvec, ldv = n;
    const int nb = W.npartial_blocks;
    double2* Vb = W.V;
    double2* Zb = W.Z;
    double2* ut = W.tmp + n;
    double2* red = W.dsmall;                 // 2m+3
    double2* h1 = red + (2 * m + 3);         // m+1
    double2* cv = h1 + (m + 1);              // m (the step records go to the pinned W.hrec)
    double2* cw = cv + m;                    // m
    double2* cu = cw + m;                    // 7: update coefficients and the scale of the candidate
    sg_solve_stats s{};
    Timer tm(c->prof.on && c->prof.mask == ~0u);
    hipEvent_t evs[2] = {nullptr, nullptr};
    SG_HIP(hipEventCreateWithFlags(&evs[0], hipEventDisableTiming));
    if (hipEventCreateWithFlags(&evs[1], hipEventDisableTiming) != hipSuccess) {
        (void)hipEventDestroy(evs[0]);
        return fail(SG_EHIP, "event creation failed");
    }
    struct EvGuard {
        hipEvent_t* e;
        ~EvGuard() {
            (void)hipEventDestroy(e[0]);
            (void)hipEventDestroy(e[1]);
        }
    } evguard{evs};

    auto norm_of = [&](const double2* v, double* out) -> int {
        int r = launch_norm2(n, v, W.partial, nb, stream);
        if (r) return r;
        if ((r = launch_reduce_norm(nb, W.partial, W.coef, stream))) return r;
        SG_HIP(hipMemcpyAsync(W.host_pinned, W.coef, sizeof(double2), hipMemcpyDeviceToHost, stream));
        if ((r = wait_stream(stream, W.done))) return r;
        *out = W.host_pinned[0].x;
        return SG_OK;
    };

    double bnorm = 0;
    if ((rc = norm_of(b, &bnorm))) return rc;
    if (!std::isfinite(bnorm)) return fail(SG_ENONFINITE, "non-finite right-hand side");
    if (o->x0_zero) SG_HIP(hipMemsetAsync(x, 0, (size_t)n * sizeof(double2), stream));
    if (bnorm == 0.0) {
        SG_HIP(hipMemsetAsync(x, 0, (size_t)n * sizeof(double2), stream));
        SG_HIP(hipStreamSynchronize(stream));
        s.converged = 1;
        s.relres_prec = 0.0;
        if (st) *st = s;
        return SG_OK;
    }
    const bool can_ahead = !tm.ok;
    bool first = true;
    int result = SG_ENOTCONV;

    while (true) {
        // r = b - A x, the candidate u_0 of slot 0 (formed in scratch first, so that a solve
        // that stops here leaves the previous cycle's basis intact)
        double beta = bnorm;
        const double2* r0 = b;
        if (!(first && o->x0_zero)) {
            tm.record(0, stream);
            if ((rc = launch_apply(c, x, ut, stream))) return rc;
            tm.record(1, stream);
            if ((rc = launch_axpby(n, make_double2(1, 0), b, make_double2(-1, 0), ut, ut, stream))) return rc;
            if ((rc = norm_of(ut, &beta))) return rc;
            s.t_matvec += tm.between(0, 1);
            r0 = ut;
        }
        first = false;
        if (!std::isfinite(beta)) return fail(SG_ENONFINITE, "non-finite residual");
        s.relres_true = beta / bnorm;
        if (s.relres_true <= o->tol) { result = SG_OK; s.converged = 1; break; }
        if (s.iters >= o->maxit) break;
        SG_HIP(hipMemcpyAsync(Vb, r0, (size_t)n * sizeof(double2), hipMemcpyDeviceToDevice, stream));

        Givens gv(m);
        gv.g[0] = beta;
        // issue step j: full (precond, operator, reduction with w, coefficients, update) or a
        // finishing reduction of u_j alone; the coefficient record goes to host buffer j & 1
        auto issue = [&](int j, bool full) -> int {
            int r;
            if (full) {
                tm.record(0, stream);
                if ((r = launch_precond(c, o->precond, o->precision, Vb + (long long)j * ldv, Zb + (long long)j * ldv,
                                        stream)))
                    return r;
                tm.record(1, stream);
                if ((r = launch_apply(c, Zb + (long long)j * ldv, Vb + (long long)(j + 1) * ldv, stream))) return r;
                tm.record(2, stream);
            }
            if ((r = launch_dcgs_reduce(n, j, Vb, ldv, Vb + (long long)j * ldv,
                                        full ? Vb + (long long)(j + 1) * ldv : nullptr, W.dpart, nb, red, stream)))
                return r;
            if ((r = launch_dcgs_finalize(j, full, red, h1, W.hrec_dev + (size_t)(j & 1) * (2 * m + 3), cv, cw, cu,
                                          stream)))
                return r;
            if (full && (r = launch_dcgs_update(n, j, Vb, ldv, Vb + (long long)j * ldv, Vb + (long long)(j + 1) * ldv,
                                                cv, cw, cu, nb, stream)))
                return r;
            SG_HIP(hipEventRecord(evs[j & 1], stream));
            if (full) tm.record(3, stream);
            return SG_OK;
        };

        int k = 0;                    // completed (committed) columns of this cycle
        bool breakdown = false, done = false;
        double est = s.relres_true;   // latest residual estimate
        int j = 0;                    // step 0 is always a full step
        bool full_j = true;
        bool queued = false;          // step j already issued (look-ahead)
        while (!done) {
            if (!queued && (rc = issue(j, full_j))) return rc;
            const bool queued_full = full_j;
            // the decisions below use the estimate known before step j's record, in both the
            // look-ahead and the profiled runs, so that both issue the same steps
            const double est_before = est;
            // look-ahead: far from the tolerance, issue step j+1 (full) before reading step j
            bool ahead = false;
            if (can_ahead && full_j && j + 1 < m && s.iters + 1 < o->maxit && est_before > 30.0 * o->tol) {
                if ((rc = issue(j + 1, true))) return rc;
                ahead = true;
            }
            if ((rc = poll(evs[j & 1]))) return rc;
            if (full_j) {
                s.t_precond += tm.between(0, 1);
                s.t_matvec += tm.between(1, 2);
                s.t_orth += tm.between(2, 3);
            }
            const double2* hr = W.hrec + (size_t)(j & 1) * (2 * m + 3);
            const double nu = hr[j].x;
            if (!std::isfinite(nu)) return fail(SG_ENONFINITE, "non-finite Arnoldi norm");
            bool finish_next = false;
            if (j >= 1 && k < j) {   // (a full step redone after a finishing one finds it committed)
                // column j-1 is complete: rows 0..j-1 from the record, row j = ν_j
                std::vector<cd> col(j + 1);
                double colnorm = 0.0;
                for (int i = 0; i < j; ++i) {
                    col[i] = cd(hr[i].x, hr[i].y);
                    if (!std::isfinite(col[i].real()) || !std::isfinite(col[i].imag()))
                        return fail(SG_ENONFINITE, "non-finite Hessenberg entry");
                    colnorm += std::norm(col[i]);
                }
                col[j] = nu;
                colnorm = std::sqrt(colnorm + nu * nu);
                const double gn = gv.add(j - 1, col, true);
                ++s.iters;
                k = j;
                est = gn / bnorm;
                s.relres_est = est;
                if (o->hist && s.iters - 1 < o->hist_cap) o->hist[s.iters - 1] = est;
                if (!(nu > 1e-14 * colnorm)) { breakdown = true; done = true; break; }
                if (est <= o->tol || s.iters >= o->maxit || j == m) { done = true; break; }
            }
            if (!queued_full) {
                // the finishing reduction did not reach the tolerance: redo step j in full
                queued = false;
                full_j = true;
                continue;
            }
            // predict column j from step j's record and decide the kind of step j+1
            if (!ahead) {
                const double pred = hr[2 * j + 2].y;
                std::vector<cd> pc(j + 2);
                for (int i = 0; i <= j; ++i) pc[i] = cd(hr[j + 1 + i].x, hr[j + 1 + i].y);
                pc[j + 1] = pred > 0.0 ? std::sqrt(pred) : 0.0;
                const double pest = gv.add(j, pc, false) / bnorm;
                finish_next = j + 1 == m || s.iters + 1 >= o->maxit || (est_before <= 30.0 * o->tol && pest <= o->tol);
            }
            ++j;
            queued = ahead;
            full_j = ahead ? true : !finish_next;
        }
        // y = R^{-1} g, x += Z y
        std::vector<cd> y(k);
        for (int i = k - 1; i >= 0; --i) {
            cd acc = gv.g[i];
            for (int l = i + 1; l < k; ++l) acc -= gv.R[(size_t)i * m + l] * y[l];
            y[i] = acc / gv.R[(size_t)i * m + i];
            if (!std::isfinite(y[i].real()) || !std::isfinite(y[i].imag()))
                return fail(SG_ENONFINITE, "non-finite least-squares solution");
        }
        // (host_pinned was last read by the residual norm of this cycle's start, whose copy
        // has completed; an unused look-ahead step writes only hrec and unused slots)
        for (int i = 0; i < k; ++i) W.host_pinned[i] = make_double2(y[i].real(), y[i].imag());
        if (k > 0) {
            SG_HIP(hipMemcpyAsync(W.coef, W.host_pinned, (size_t)k * sizeof(double2), hipMemcpyHostToDevice, stream));
            if ((rc = launch_lincomb(n, k, Zb, ldv, nullptr, W.coef, x, stream))) return rc;
        }
        ++s.restarts;
        c->last_k = k;
        if (breakdown) {
            if ((rc = launch_apply(c, x, ut, stream))) return rc;
            if ((rc = launch_axpby(n, make_double2(1, 0), b, make_double2(-1, 0), ut, ut, stream))) return rc;
            double rn = 0;
            if ((rc = norm_of(ut, &rn))) return rc;
            s.relres_true = rn / bnorm;
            if (s.relres_true <= o->tol) { result = SG_OK; s.converged = 1; }
            else result = SG_EBREAKDOWN;
            break;
        }
    }
    s.relres_prec = s.relres_true;
    s.t_setup = c->t_setup_ms;
    s.t_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (st) *st = s;
    if (result == SG_EBREAKDOWN) return fail(SG_EBREAKDOWN, "breakdown before reaching the tolerance");
    return result;
}

}  // namespace sgi
