// Restarted right-preconditioned GMRES(m) and flexible GMRES(m) drivers.
//
// Right preconditioning solves A P^{-1} y = b, x = P^{-1} y, so the residual that is
// monitored is the one of the unpreconditioned system, ||b - Ax||/||b|| (eq.
// CSL_preconditioned, eq. preconditioned_2d, Section 6.3).  Each Arnoldi step:
//   z_j = P^{-1} v_j            (sg_precond or a user callback)
//   w   = A z_j                 (sg_apply)
//   CGS2: h = Vᴴw, w -= Vh, twice; h_{j+1,j} = ||w||    (classical Gram-Schmidt with
//         one full re-orthogonalisation)
//   complex Givens rotation of the new Hessenberg column, |g_{j+1}|/||b|| estimate.
// A cycle ends at the estimate tolerance, at m steps or at breakdown; x is updated
// (x += P^{-1} V y, or x += Z y for the flexible form) and the true FP64 residual
// decides between stopping and restarting.  Basis vectors are stored unnormalised
// with a per-vector scale (v_k = s_k V_k).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "sg_internal.h"

namespace sgi {

int ensure_workspace(Ctx* c, int m, bool flexible) {
    Workspace& w = c->ws;
    if (w.V && w.done && w.m >= m && (!flexible || w.Z)) return SG_OK;   // w.done is set last
    (void)hipFree(w.V);
    (void)hipFree(w.Z);
    (void)hipFree(w.tmp);
    (void)hipFree(w.scale);
    (void)hipFree(w.coef);
    (void)hipFree(w.partial);
    if (w.host_pinned) (void)hipHostFree(w.host_pinned);
    if (w.done) (void)hipEventDestroy(w.done);
    (void)hipFree(w.dpart);
    (void)hipFree(w.dsmall);
    if (w.hrec) (void)hipHostFree(w.hrec);
    w = Workspace{};
    const size_t nv = (size_t)c->nvec;
    w.m = m;
    w.flexible = flexible;
    w.npartial_blocks = reduction_blocks(c->nvec);
    if (device_alloc((void**)&w.V, (size_t)(m + 1) * nv * sizeof(double2)) != hipSuccess)
        return fail(SG_ENOMEM, "Krylov basis allocation failed");
    if (flexible && device_alloc((void**)&w.Z, (size_t)m * nv * sizeof(double2)) != hipSuccess)
        return fail(SG_ENOMEM, "flexible basis allocation failed");
    if (device_alloc((void**)&w.tmp, 2 * nv * sizeof(double2)) != hipSuccess)
        return fail(SG_ENOMEM, "scratch allocation failed");
    SG_HIP(hipMalloc(&w.scale, (size_t)(m + 2) * sizeof(double)));
    SG_HIP(hipMalloc(&w.coef, (size_t)3 * (m + 2) * sizeof(double2)));
    SG_HIP(hipMalloc(&w.partial, (size_t)w.npartial_blocks * (m + 2) * sizeof(double2)));
    SG_HIP(hipHostMalloc(&w.host_pinned, (size_t)3 * (m + 2) * sizeof(double2), hipHostMallocDefault));
    SG_HIP(hipEventCreateWithFlags(&w.done, hipEventDisableTiming));
    return SG_OK;
}

// Spin until ev has completed.
static int poll_event(hipEvent_t ev) {
    hipError_t e;
    while ((e = hipEventQuery(ev)) == hipErrorNotReady) {
    }
    SG_HIP(e);
    return SG_OK;
}

// Wait until the work queued on st has finished.  With an event the host polls it (the
// waits of the Arnoldi loop are a few hundred microseconds apart, and a blocking wait
// adds tens of microseconds of wake-up latency to each); without one, a blocking wait.
int wait_stream(hipStream_t st, hipEvent_t ev) {
    if (!ev) {
        SG_HIP(hipStreamSynchronize(st));
        return SG_OK;
    }
    SG_HIP(hipEventRecord(ev, st));
    return poll_event(ev);
}

// Two passes of classical Gram-Schmidt of w against v_k = s_k V_k (k < nv), then ||w||.
// On return h_pinned[0..nv) = pass-1 coefficients, [nv..2nv) = pass-2 coefficients,
// h_pinned[2nv].x = ||w|| after both passes; the stream is synchronised (or, with
// wait = false, `done` is recorded after the copy and the caller polls it).  The
// reciprocal norm, the lazy scale of the next basis vector, is also left in d_next_scale on
// the device, so that the next step needs no host-to-device copy.
int cgs2_step(long long n, int nv, const double2* V, long long ldv, const double* d_scale, double2* w,
              double2* partial, int nblocks, double2* d_coef, double2* h_pinned, hipStream_t st,
              double* d_next_scale, hipEvent_t done, bool wait) {
    int rc;
    // pass 1 projection
    if ((rc = launch_multidot(n, nv, V, ldv, d_scale, w, partial, nblocks, st))) return rc;
    if ((rc = launch_reduce(nblocks, nv, partial, d_scale, d_coef, st))) return rc;
    // pass 1 update fused with the pass 2 projection, pass 2 update fused with the norm
    int fused = launch_upd(n, nv, V, ldv, d_scale, d_coef, w, partial, nblocks, true, st);
    if (fused < 0) return fused;
    if (fused) {
        if ((rc = launch_reduce(nblocks, nv, partial, d_scale, d_coef + nv, st))) return rc;
        if ((rc = launch_upd(n, nv, V, ldv, d_scale, d_coef + nv, w, partial, nblocks, false, st)) < 0) return rc;
    } else {
        if ((rc = launch_axpy_dot(n, nv, V, ldv, d_scale, d_coef, w, nullptr, 0, false, st))) return rc;
        if ((rc = launch_multidot(n, nv, V, ldv, d_scale, w, partial, nblocks, st))) return rc;
        if ((rc = launch_reduce(nblocks, nv, partial, d_scale, d_coef + nv, st))) return rc;
        if ((rc = launch_axpy_dot(n, nv, V, ldv, d_scale, d_coef + nv, w, nullptr, 0, false, st))) return rc;
        if ((rc = launch_norm2(n, w, partial, nblocks, st))) return rc;
    }
    if ((rc = launch_reduce_norm(nblocks, partial, d_coef + 2 * nv, st, d_next_scale))) return rc;
    SG_HIP(hipMemcpyAsync(h_pinned, d_coef, (size_t)(2 * nv + 1) * sizeof(double2), hipMemcpyDeviceToHost, st));
    if (!wait && done) {
        SG_HIP(hipEventRecord(done, st));
        return SG_OK;
    }
    return wait_stream(st, done);
}

// ||x|| to the host; d_inv (device, may be null) also receives 1/||x||.
static int norm_sync(Ctx* c, const double2* x, double* out, hipStream_t st, double* d_inv = nullptr) {
    Workspace& w = c->ws;
    int rc = launch_norm2(c->nvec, x, w.partial, w.npartial_blocks, st);
    if (rc) return rc;
    if ((rc = launch_reduce_norm(w.npartial_blocks, w.partial, w.coef, st, d_inv))) return rc;
    SG_HIP(hipMemcpyAsync(w.host_pinned, w.coef, sizeof(double2), hipMemcpyDeviceToHost, st));
    if ((rc = wait_stream(st, w.done))) return rc;
    *out = w.host_pinned[0].x;
    return SG_OK;
}

namespace {
// Per-phase timing of the solve statistics, recorded only while the handle's profiler is
// on: an event between two kernels leaves the GPU idle for a few microseconds.
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
}  // namespace

int run_gmres(Ctx* c, const double2* b, double2* x, const sg_solve_opts* o, sg_precond_cb cb, void* user,
              bool flexible, sg_solve_stats* st, hipStream_t stream) {
    using cd = std::complex<double>;
    auto t_start = std::chrono::steady_clock::now();
    if (!o || !b || !x) return fail(SG_EINVAL, "null argument");
    if (o->restart < 1 || o->restart > 512) return fail(SG_EINVAL, "restart must be in [1, 512]");
    if (o->maxit < 1) return fail(SG_EINVAL, "maxit must be >= 1");
    if (!(o->tol > 0)) return fail(SG_EINVAL, "tol must be positive");
    if (!cb && (o->precond < SG_PC_NONE || o->precond > SG_PC_MEAN_NET))
        return fail(SG_EINVAL, "unsupported built-in preconditioner");
    if (!cb && o->precond == SG_PC_MEAN_NET && (!c->net || !flexible))
        return fail(SG_EINVAL, "the learned preconditioner needs an attached network and flexible GMRES");
    if (o->side != 0 && o->side != 1) return fail(SG_EINVAL, "side must be 0 (right) or 1 (left)");
    const bool left = o->side == 1;
    if (left && (flexible || cb || o->precond == SG_PC_MEAN_NET))
        return fail(SG_EINVAL, "left preconditioning is available in sg_gmres with a built-in preconditioner");
    const int m = o->restart;
    int rc = ensure_workspace(c, m, flexible);
    if (rc) return rc;
    Workspace& W = c->ws;
    const long long n = c->nvec;
    const long long ldv = n;
    sg_solve_stats s{};
    Timer tm(c->prof.on && c->prof.mask == ~0u);   // phase times only under full profiling

    auto precond = [&](const double2* in, double2* out) -> int {
        if (cb) {
            int r = cb(user, reinterpret_cast<const sg_c64*>(in), reinterpret_cast<sg_c64*>(out), stream);
            return r == 0 ? SG_OK : fail(SG_EINVAL, "preconditioner callback returned " + std::to_string(r));
        }
        if (o->precond == SG_PC_MEAN_NET) return net_precond(c->net, c, o->precision, in, out, stream);
        return launch_precond(c, o->precond, o->precision, in, out, stream);
    };

    double bnorm = 0;
    // from x = 0 the first residual is b itself (right) or P^{-1} b (left): its norm and lazy
    // scale serve the first cycle
    if ((rc = norm_sync(c, b, &bnorm, stream, (o->x0_zero && !left) ? W.scale : nullptr))) return rc;
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
    // Left preconditioning (eq. CSL_preconditioned, second system): the residual is the
    // preconditioned one (Section 6.3), so the relative test uses ||P^{-1} b||.
    double pbnorm = bnorm;
    if (left) {
        if ((rc = precond(b, W.tmp))) return rc;
        if ((rc = norm_sync(c, W.tmp, &pbnorm, stream, o->x0_zero ? W.scale : nullptr))) return rc;
        if (!std::isfinite(pbnorm)) return fail(SG_ENONFINITE, "non-finite preconditioned right-hand side");
        if (pbnorm == 0.0) return fail(SG_EBREAKDOWN, "the preconditioned right-hand side is zero");
    }
    const double rden = left ? pbnorm : bnorm;
    // The preconditioner and operator of Arnoldi step j+1 need no host result (the lazy
    // scale of v_{j+1} is formed on the device), so with the built-in preconditioners they
    // are queued before the host waits for step j's coefficients, hiding the host's turn
    // (wait, least-squares update, launches).  It is done while the estimate is above
    // 30·tol, so the work rarely goes unused; unused, it only writes buffers that the
    // cycle's update does not read.  Not under full profiling, whose phase times need the
    // phases apart.
    const bool can_ahead = !cb && o->precond != SG_PC_MEAN_NET && !tm.ok;
    double2* Vb = W.V;
    double2* zt = W.tmp;            // z_j (non-flexible) / update scratch
    double2* ut = W.tmp + n;
    std::vector<double> hscale(m + 2, 1.0);
    std::vector<cd> H((size_t)(m + 1) * m), R((size_t)(m + 1) * m), g(m + 1), sn(m);
    std::vector<double> cs(m);
    bool first = true;
    int result = SG_ENOTCONV;

    while (true) {
        // r = b - A x (left: P^{-1}(b - A x)), stored as V_0
        if (first && o->x0_zero) {
            SG_HIP(hipMemcpyAsync(Vb, left ? W.tmp : b, (size_t)n * sizeof(double2), hipMemcpyDeviceToDevice, stream));
        } else {
            tm.record(0, stream);
            if ((rc = launch_apply(c, x, ut, stream))) return rc;
            tm.record(1, stream);
            if ((rc = launch_axpby(n, make_double2(1, 0), b, make_double2(-1, 0), ut, left ? ut : Vb, stream)))
                return rc;
            if (left && (rc = precond(ut, Vb))) return rc;
        }
        double beta = rden;
        if (!(first && o->x0_zero) && (rc = norm_sync(c, Vb, &beta, stream, W.scale)))   // W.scale[0] = 1/beta
            return rc;
        if (!(first && o->x0_zero)) s.t_matvec += tm.between(0, 1);
        first = false;
        if (!std::isfinite(beta)) return fail(SG_ENONFINITE, "non-finite residual");
        if (left) s.relres_prec = beta / rden;
        else s.relres_true = beta / bnorm;
        if (beta / rden <= o->tol) { result = SG_OK; s.converged = 1; break; }
        if (s.iters >= o->maxit) break;
        hscale[0] = 1.0 / beta;   // the same value the device stored in W.scale[0]
        std::fill(g.begin(), g.end(), cd(0));
        g[0] = beta;
        int k = 0;
        bool breakdown = false;
        bool queued = false;                 // step j's preconditioner and operator already queued
        double est_prev = s.relres_true;     // latest residual estimate
        auto queue_pa = [&](int jj) -> int {   // w_{jj+1} = A P^{-1} V_jj (left: P^{-1} A V_jj), unscaled
            if (left) {
                int r2 = launch_apply(c, Vb + (long long)jj * ldv, ut, stream);
                if (r2) return r2;
                tm.record(1, stream);
                return precond(ut, Vb + (long long)(jj + 1) * ldv);
            }
            double2* zz = flexible ? W.Z + (long long)jj * ldv : zt;
            int r2 = precond(Vb + (long long)jj * ldv, zz);
            if (r2) return r2;
            tm.record(1, stream);
            return launch_apply(c, zz, Vb + (long long)(jj + 1) * ldv, stream);
        };
        for (int j = 0; j < m; ++j) {
            double2* wv = Vb + (long long)(j + 1) * ldv;
            tm.record(0, stream);
            if (!queued && (rc = queue_pa(j))) return rc;
            tm.record(2, stream);
            const bool ahead = can_ahead && j + 1 < m && s.iters + 1 < o->maxit && est_prev > 30.0 * o->tol;
            if ((rc = cgs2_step(n, j + 1, Vb, ldv, W.scale, wv, W.partial, W.npartial_blocks, W.coef,
                                W.host_pinned, stream, W.scale + j + 1, W.done, !ahead)))
                return rc;
            if (ahead) {
                if ((rc = queue_pa(j + 1))) return rc;
                if ((rc = poll_event(W.done))) return rc;
            }
            queued = ahead;
            tm.record(3, stream);
            s.t_precond += tm.between(0, 1);
            s.t_matvec += tm.between(1, 2);
            s.t_orth += tm.between(2, 3);
            const double sj = hscale[j];
            double colnorm = 0;
            for (int i = 0; i <= j; ++i) {
                const double2 a1 = W.host_pinned[i], a2 = W.host_pinned[j + 1 + i];
                const cd hv = sj * cd(a1.x + a2.x, a1.y + a2.y);
                if (!std::isfinite(hv.real()) || !std::isfinite(hv.imag()))
                    return fail(SG_ENONFINITE, "non-finite Hessenberg entry");
                H[(size_t)i * m + j] = hv;
                colnorm += std::norm(hv);
            }
            const double nrm = W.host_pinned[2 * (j + 1)].x;
            if (!std::isfinite(nrm)) return fail(SG_ENONFINITE, "non-finite Arnoldi norm");
            const double hnext = sj * nrm;
            H[(size_t)(j + 1) * m + j] = hnext;
            colnorm = std::sqrt(colnorm + hnext * hnext);
            // apply previous rotations to column j, then a new one
            std::vector<cd> col(j + 2);
            for (int i = 0; i <= j + 1; ++i) col[i] = H[(size_t)i * m + j];
            for (int i = 0; i < j; ++i) {
                const cd t = cs[i] * col[i] + sn[i] * col[i + 1];
                col[i + 1] = -std::conj(sn[i]) * col[i] + cs[i] * col[i + 1];
                col[i] = t;
            }
            const cd a = col[j], bb = col[j + 1];
            double cj;
            cd sjr;
            if (std::abs(bb) == 0.0) { cj = 1.0; sjr = 0.0; }
            else if (std::abs(a) == 0.0) { cj = 0.0; sjr = std::conj(bb) / std::abs(bb); }
            else {
                const double t = std::hypot(std::abs(a), std::abs(bb));
                cj = std::abs(a) / t;
                sjr = (a / std::abs(a)) * std::conj(bb) / t;
            }
            cs[j] = cj;
            sn[j] = sjr;
            col[j] = cj * a + sjr * bb;
            col[j + 1] = 0.0;
            for (int i = 0; i <= j + 1; ++i) R[(size_t)i * m + j] = col[i];
            g[j + 1] = -std::conj(sjr) * g[j];
            g[j] = cj * g[j];
            ++s.iters;
            k = j + 1;
            s.relres_est = std::abs(g[j + 1]) / rden;
            est_prev = s.relres_est;
            if (o->hist && s.iters - 1 < o->hist_cap) o->hist[s.iters - 1] = s.relres_est;
            if (!(nrm > 1e-14 * colnorm / (sj > 0 ? sj : 1.0)) || hnext <= 1e-14 * colnorm) { breakdown = true; break; }
            hscale[j + 1] = 1.0 / nrm;   // the same value cgs2_step left in W.scale[j + 1]
            if (nrm > 1e50 || nrm < 1e-50) {
                // The stored vectors are unnormalised (lazy scales), so each step multiplies their
                // size by about ||A P^{-1}||; store V_{j+1} normalised before that overflows
                // (or underflows) the squared sums, together with what was already formed from
                // it by the look-ahead (w_{j+2} and, flexible, Z_{j+1}), and make its scale 1.
                const double inv = hscale[j + 1];
                if ((rc = launch_scale_copy(n, inv, wv, wv, stream))) return rc;
                if (queued) {
                    double2* wn = Vb + (long long)(j + 2) * ldv;
                    if ((rc = launch_scale_copy(n, inv, wn, wn, stream))) return rc;
                    if (flexible) {
                        double2* zn = W.Z + (long long)(j + 1) * ldv;
                        if ((rc = launch_scale_copy(n, inv, zn, zn, stream))) return rc;
                    }
                }
                static const double one = 1.0;
                SG_HIP(hipMemcpyAsync(W.scale + j + 1, &one, sizeof(double), hipMemcpyHostToDevice, stream));
                hscale[j + 1] = 1.0;
            }
            if (s.relres_est <= o->tol || s.iters >= o->maxit) break;
        }
        // y = R^{-1} g (upper triangular k×k)
        std::vector<cd> y(k);
        for (int i = k - 1; i >= 0; --i) {
            cd acc = g[i];
            for (int l = i + 1; l < k; ++l) acc -= R[(size_t)i * m + l] * y[l];
            y[i] = acc / R[(size_t)i * m + i];
            if (!std::isfinite(y[i].real()) || !std::isfinite(y[i].imag()))
                return fail(SG_ENONFINITE, "non-finite least-squares solution");
        }
        for (int i = 0; i < k; ++i) W.host_pinned[i] = make_double2(y[i].real(), y[i].imag());
        SG_HIP(hipMemcpyAsync(W.coef, W.host_pinned, (size_t)k * sizeof(double2), hipMemcpyHostToDevice, stream));
        if (left) {
            if ((rc = launch_lincomb(n, k, Vb, ldv, W.scale, W.coef, x, stream))) return rc;   // x += V y
        } else if (flexible) {
            // z_j = P^{-1}(s_j V_j) was formed from the unscaled V_j: the same lazy scales
            // W.scale[0..k) apply to Z
            if ((rc = launch_lincomb(n, k, W.Z, ldv, W.scale, W.coef, x, stream))) return rc;
        } else {
            SG_HIP(hipMemsetAsync(ut, 0, (size_t)n * sizeof(double2), stream));
            if ((rc = launch_lincomb(n, k, Vb, ldv, W.scale, W.coef, ut, stream))) return rc;
            if ((rc = precond(ut, zt))) return rc;
            if ((rc = launch_axpby(n, make_double2(1, 0), x, make_double2(1, 0), zt, x, stream))) return rc;
        }
        // (the coefficients went up from pinned memory, which the host does not touch again
        // before the next wait, so no wait is needed here)
        ++s.restarts;
        if (breakdown) {
            // the Krylov space is invariant: the update is the solution of this space
            tm.record(0, stream);
            if ((rc = launch_apply(c, x, ut, stream))) return rc;
            if ((rc = launch_axpby(n, make_double2(1, 0), b, make_double2(-1, 0), ut, ut, stream))) return rc;
            if (left && (rc = precond(ut, zt))) return rc;
            double rn = 0;
            if ((rc = norm_sync(c, left ? zt : ut, &rn, stream))) return rc;
            if (left) s.relres_prec = rn / rden;
            else s.relres_true = rn / bnorm;
            if (rn / rden <= o->tol) { result = SG_OK; s.converged = 1; }
            else result = SG_EBREAKDOWN;
            break;
        }
    }
    if (left) {   // the unpreconditioned residual of the final iterate, reported beside it
        if ((rc = launch_apply(c, x, ut, stream))) return rc;
        if ((rc = launch_axpby(n, make_double2(1, 0), b, make_double2(-1, 0), ut, ut, stream))) return rc;
        double rn = 0;
        if ((rc = norm_sync(c, ut, &rn, stream))) return rc;
        s.relres_true = rn / bnorm;
    } else {
        s.relres_prec = s.relres_true;
    }
    s.t_setup = c->t_setup_ms;
    s.t_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (st) *st = s;
    if (result == SG_EBREAKDOWN) return fail(SG_EBREAKDOWN, "breakdown before reaching the tolerance");
    return result;
}

// Stationary iteration B x_{i+1} = b - (A - B) x_i from x_0 = B^{-1} b (eq.
// stationary_iteration), written as the correction x_{i+1} = x_i + B^{-1}(b - A x_i).
int run_stationary(Ctx* c, const double2* b, double2* x, int pc, int iters, double* hist, hipStream_t st) {
    if (!b || !x) return fail(SG_EINVAL, "null argument");
    if (b == x) return fail(SG_EINVAL, "sg_stationary: b and x must not alias");
    if (pc != SG_PC_MEAN && pc != SG_PC_CSL_MEAN) return fail(SG_EINVAL, "sg_stationary: pc must be a mean-based block preconditioner");
    if (iters < 0) return fail(SG_EINVAL, "sg_stationary: iters must be >= 0");
    int rc = ensure_workspace(c, 1, false);
    if (rc) return rc;
    const long long n = c->nvec;
    double2* r = c->ws.tmp;
    double2* z = c->ws.tmp + n;
    const double2 one = make_double2(1.0, 0.0), mone = make_double2(-1.0, 0.0);
    double bnorm = 0.0;
    if ((rc = norm_sync(c, b, &bnorm, st))) return rc;
    if (bnorm == 0.0) {
        if ((rc = launch_scale_copy(n, 0.0, b, x, st))) return rc;
        if (hist)
            for (int i = 0; i <= iters; ++i) hist[i] = 0.0;
        return wait_stream(st, c->ws.done);
    }
    if ((rc = launch_precond(c, pc, SG_PREC_F64, b, x, st))) return rc;
    for (int i = 0; i <= iters; ++i) {
        const bool last = i == iters;
        if (hist || !last) {
            if ((rc = launch_apply(c, x, r, st))) return rc;
            if ((rc = launch_axpby(n, one, b, mone, r, r, st))) return rc;   // r = b - A x_i
        }
        if (hist) {
            double rn = 0.0;
            if ((rc = norm_sync(c, r, &rn, st))) return rc;
            hist[i] = rn / bnorm;
            if (!std::isfinite(hist[i])) return fail(SG_ENONFINITE, "sg_stationary: the iteration diverged to a non-finite residual");
        }
        if (last) break;
        if ((rc = launch_precond(c, pc, SG_PREC_F64, r, z, st))) return rc;
        if ((rc = launch_axpby(n, one, x, one, z, x, st))) return rc;        // x_{i+1} = x_i + B^{-1} r
    }
    return SG_OK;
}

}  // namespace sgi
