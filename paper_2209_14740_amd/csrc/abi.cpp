// extern "C" entry points of include/sg.h.  Every function converts C++ exceptions
// into status codes; none aborts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "net_internal.h"
#include "sg_internal.h"

using sgi::Ctx;
using sgi::fail;

static Ctx* ctx(sg_handle h) { return reinterpret_cast<Ctx*>(h); }

static int guard_device(Ctx* c) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SG_EHIP, "hipGetDevice failed");
    if (dev != c->device) return fail(SG_EINVAL, "handle was created on another device");
    return SG_OK;
}

// Makes the handle's profiler the current one for the duration of an entry point.
struct ProfBind {
    sgi::Prof* prev;
    explicit ProfBind(Ctx* c) : prev(sgi::g_prof) { sgi::g_prof = &c->prof; }
    ~ProfBind() { sgi::g_prof = prev; }
};

#define SG_TRY(...)                                                        \
    try {                                                                  \
        __VA_ARGS__                                                        \
    } catch (const std::bad_alloc&) {                                      \
        return fail(SG_ENOMEM, "host allocation failed");                  \
    } catch (...) {                                                        \
        return fail(SG_EINVAL, "unexpected exception");                    \
    }

extern "C" {

int sg_setup(const sg_problem* prob, hipStream_t stream, sg_handle* out) {
    SG_TRY({
        if (!out) return fail(SG_EINVAL, "out is null");
        *out = nullptr;
        Ctx* c = nullptr;
        int rc = sgi::build_ctx(prob, stream, &c);
        if (rc != SG_OK) return rc;
        *out = reinterpret_cast<sg_handle>(c);
        return SG_OK;
    })
}

void sg_destroy(sg_handle h) {
    try {
        delete ctx(h);
    } catch (...) {
    }
}

int sg_basis(sg_handle h, int* Q, int* multi_index) {
    SG_TRY({
        if (!h || !Q) return fail(SG_EINVAL, "null argument");
        Ctx* c = ctx(h);
        *Q = c->Q;
        if (multi_index)
            for (size_t i = 0; i < c->alpha.size(); ++i) multi_index[i] = c->alpha[i];
        return SG_OK;
    })
}

long long sg_size(sg_handle h) { return h ? ctx(h)->nvec : 0; }

int sg_rhs(sg_handle h, const double* f_host, sg_c64* b_dev, hipStream_t stream) {
    SG_TRY({
        if (!h || !f_host || !b_dev) return fail(SG_EINVAL, "null argument");
        Ctx* c = ctx(h);
        if (int rc = guard_device(c)) return rc;
        const std::vector<double>& w = c->w_host;
        std::vector<double2> b0(c->P);
        for (long long i = 0; i < c->P; ++i) b0[i] = make_double2(w[i] * f_host[i], 0.0);
        SG_HIP(hipMemsetAsync(b_dev, 0, (size_t)c->nvec * sizeof(double2), stream));
        SG_HIP(hipMemcpyAsync(b_dev, b0.data(), (size_t)c->P * sizeof(double2), hipMemcpyHostToDevice, stream));
        SG_HIP(hipStreamSynchronize(stream));
        return SG_OK;
    })
}

int sg_apply(sg_handle h, const sg_c64* x, sg_c64* y, hipStream_t stream) {
    SG_TRY({
        if (!h || !x || !y) return fail(SG_EINVAL, "null argument");
        Ctx* c = ctx(h);
        if (int rc = guard_device(c)) return rc;
        ProfBind pb(c);
        return sgi::launch_apply(c, reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y), stream);
    })
}

int sg_moments(sg_handle h, const sg_c64* x, sg_c64* mean, double* var, hipStream_t stream) {
    SG_TRY({
        if (!h || !x || (!mean && !var)) return fail(SG_EINVAL, "null argument");
        Ctx* c = ctx(h);
        if (int rc = guard_device(c)) return rc;
        ProfBind pb(c);
        return sgi::launch_moments(c, reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(mean), var,
                                   stream);
    })
}

int sg_degree_magnitudes(sg_handle h, const sg_c64* x, double* gamma_host, hipStream_t stream) {
    SG_TRY({
        if (!h || !x || !gamma_host) return fail(SG_EINVAL, "null argument");
        Ctx* c = ctx(h);
        if (int rc = guard_device(c)) return rc;
        return sgi::degree_magnitudes(c, reinterpret_cast<const double2*>(x), gamma_host, stream);
    })
}

int sg_set_orthogonalisation(sg_handle h, int kind) {
    SG_TRY({
        if (!h) return fail(SG_EINVAL, "null handle");
        if (kind != SG_ORTH_DCGS2 && kind != SG_ORTH_CGS2) return fail(SG_EINVAL, "unknown orthogonalisation");
        ctx(h)->classic_cgs2 = kind == SG_ORTH_CGS2;
        return SG_OK;
    })
}

int sg_last_basis(sg_handle h, int* nvec, const sg_c64** V) {
    SG_TRY({
        if (!h || !nvec || !V) return fail(SG_EINVAL, "null argument");
        Ctx* c = ctx(h);
        *nvec = c->last_k;
        *V = reinterpret_cast<const sg_c64*>(c->ws.V);
        return SG_OK;
    })
}

int sg_set_eigen_cond_limit(double limit) {
    SG_TRY({
        if (!(limit >= 1.0)) return fail(SG_EINVAL, "sg_set_eigen_cond_limit: limit must be >= 1");
        sgi::set_eigen_cond_limit(limit);
        return SG_OK;
    })
}

int sg_mean_solver(sg_handle h, int* kind, double* cond_v) {
    SG_TRY({
        if (!h) return fail(SG_EINVAL, "null handle");
        Ctx* c = ctx(h);
        if (kind) *kind = !c->vmean ? SG_MEAN_FD : (c->eig_fallback ? SG_MEAN_LINE_FALLBACK : SG_MEAN_LINE);
        if (cond_v) *cond_v = c->cond_v;
        return SG_OK;
    })
}

int sg_setup_times(sg_handle h, double* ms) {
    SG_TRY({
        if (!h || !ms) return fail(SG_EINVAL, "null argument");
        const Ctx* c = ctx(h);
        ms[0] = c->t_setup_ms;
        ms[1] = c->t_setup_alloc_ms;
        ms[2] = c->t_setup_upload_ms;
        ms[3] = c->t_setup_stream_ms;
        return SG_OK;
    })
}

int sg_set_operator_shift(sg_handle h, double beta) {
    SG_TRY({
        if (!h) return fail(SG_EINVAL, "null handle");
        if (!std::isfinite(beta)) return fail(SG_EINVAL, "sg_set_operator_shift: beta must be finite");
        if (beta != 0.0 && !sgi::apply_available(ctx(h), beta))
            return fail(SG_EINVAL, "sg_set_operator_shift: no operator kernel serves the shifted operator of this shape");
        ctx(h)->op_csl_beta = beta;
        return SG_OK;
    })
}

int sg_precond(sg_handle h, int pc, int precision, const sg_c64* r, sg_c64* z, hipStream_t stream) {
    SG_TRY({
        if (!h || !r || !z) return fail(SG_EINVAL, "null argument");
        Ctx* c = ctx(h);
        if (int rc = guard_device(c)) return rc;
        ProfBind pb(c);
        if (pc == SG_PC_MEAN_NET) {
            if (!c->net) return fail(SG_EINVAL, "sg_precond: no network attached");
            if (precision < SG_PREC_F64 || precision > SG_PREC_BF16X3) return fail(SG_EINVAL, "unknown precision");
            return sgi::net_precond(c->net, c, precision, reinterpret_cast<const double2*>(r),
                                    reinterpret_cast<double2*>(z), stream);
        }
        return sgi::launch_precond(c, pc, precision, reinterpret_cast<const double2*>(r),
                                   reinterpret_cast<double2*>(z), stream);
    })
}

int sg_gmres(sg_handle h, const sg_c64* b, sg_c64* x, const sg_solve_opts* opts, sg_solve_stats* stats,
             hipStream_t stream) {
    SG_TRY({
        if (!h) return fail(SG_EINVAL, "null handle");
        Ctx* c = ctx(h);
        if (int rc = guard_device(c)) return rc;
        ProfBind pb(c);
        if (sgi::dcgs2_serves(c, opts, nullptr) && !c->classic_cgs2) {
            const int rc = sgi::run_gmres_dcgs2(c, reinterpret_cast<const double2*>(b), reinterpret_cast<double2*>(x),
                                                opts, stats, stream);
            // the delayed form keeps a flexible basis (2m+1 vectors); when it does not fit, the
            // two-pass driver solves with m+1
            if (rc != SG_ENOMEM) return rc;
        }
        return sgi::run_gmres(c, reinterpret_cast<const double2*>(b), reinterpret_cast<double2*>(x), opts, nullptr,
                              nullptr, false, stats, stream);
    })
}

int sg_stationary(sg_handle h, const sg_c64* b, sg_c64* x, int pc, int iters, double* hist, hipStream_t stream) {
    SG_TRY({
        if (!h) return fail(SG_EINVAL, "null handle");
        Ctx* c = ctx(h);
        if (int rc = guard_device(c)) return rc;
        ProfBind pb(c);
        return sgi::run_stationary(c, reinterpret_cast<const double2*>(b), reinterpret_cast<double2*>(x), pc, iters,
                                   hist, stream);
    })
}

int sg_fgmres(sg_handle h, const sg_c64* b, sg_c64* x, const sg_solve_opts* opts, sg_precond_cb cb, void* user,
              sg_solve_stats* stats, hipStream_t stream) {
    SG_TRY({
        if (!h) return fail(SG_EINVAL, "null handle");
        Ctx* c = ctx(h);
        if (int rc = guard_device(c)) return rc;
        ProfBind pb(c);
        const double2* bb = reinterpret_cast<const double2*>(b);
        double2* xx = reinterpret_cast<double2*>(x);
        if (sgi::dcgs2_serves(c, opts, cb) && !c->classic_cgs2)
            return sgi::run_gmres_dcgs2(c, bb, xx, opts, stats, stream);
        if (cb || !opts || opts->precond != SG_PC_MEAN_NET)
            return sgi::run_gmres(c, bb, xx, opts, cb, user, true, stats, stream);
        if (!c->net) return fail(SG_EINVAL, "sg_fgmres: no network attached");
        // one cycle of FGMRES with the learned preconditioner
        sg_solve_opts o1 = *opts;
        o1.maxit = std::min(opts->maxit, opts->restart);
        sg_solve_stats s1{};
        int rc = sgi::run_gmres(c, bb, xx, &o1, nullptr, nullptr, true, &s1, stream);
        if (rc == SG_OK) {
            if (stats) *stats = s1;
            return SG_OK;
        }
        if (rc < 0 && rc != SG_ENONFINITE && rc != SG_EBREAKDOWN) return rc;
        // fallback: plain A_0-preconditioned GMRES, warm-started when the iterate is usable
        const bool warm = rc == SG_ENOTCONV && std::isfinite(s1.relres_true) && s1.relres_true < 1.0;
        sg_solve_opts o2 = *opts;
        o2.precond = SG_PC_MEAN;
        o2.x0_zero = warm ? 0 : 1;
        o2.maxit = std::max(1, opts->maxit - s1.iters);
        o2.hist = opts->hist && opts->hist_cap > s1.iters ? opts->hist + s1.iters : nullptr;
        o2.hist_cap = o2.hist ? opts->hist_cap - s1.iters : 0;
        sg_solve_stats s2{};
        rc = sgi::run_gmres(c, bb, xx, &o2, nullptr, nullptr, false, &s2, stream);
        s2.iters += s1.iters;
        s2.restarts += s1.restarts;
        s2.fallback = 1;
        s2.t_precond += s1.t_precond;
        s2.t_matvec += s1.t_matvec;
        s2.t_orth += s1.t_orth;
        s2.t_total += s1.t_total;
        if (stats) *stats = s2;
        return rc == SG_OK ? SG_FALLBACK_USED : rc;
    })
}

int sg_cgs2(long long n, int nv, const sg_c64* V, sg_c64* w, sg_c64* h_host, hipStream_t stream) {
    SG_TRY({
        if (n < 1 || nv < 1 || nv > 512 || !V || !w || !h_host) return fail(SG_EINVAL, "invalid argument");
        const int nb = sgi::reduction_blocks(n);
        double2 *partial = nullptr, *coef = nullptr, *pin = nullptr;
        int rc = SG_OK;
        if (hipMalloc(&partial, (size_t)nb * (nv + 1) * sizeof(double2)) != hipSuccess ||
            hipMalloc(&coef, (size_t)(2 * nv + 2) * sizeof(double2)) != hipSuccess ||
            hipHostMalloc(&pin, (size_t)(2 * nv + 2) * sizeof(double2), hipHostMallocDefault) != hipSuccess) {
            rc = fail(SG_ENOMEM, "sg_cgs2 scratch allocation failed");
        } else {
            rc = sgi::cgs2_step(n, nv, reinterpret_cast<const double2*>(V), n, nullptr, reinterpret_cast<double2*>(w),
                                partial, nb, coef, pin, stream);
            if (rc == SG_OK) {
                const double nrm = pin[2 * nv].x;
                for (int k = 0; k < nv; ++k)
                    h_host[k] = sg_c64{pin[k].x + pin[nv + k].x, pin[k].y + pin[nv + k].y};
                h_host[nv] = sg_c64{nrm, 0.0};
                if (!std::isfinite(nrm)) rc = fail(SG_ENONFINITE, "non-finite norm");
                else if (nrm > 0.0) {
                    rc = sgi::launch_scale_copy(n, 1.0 / nrm, reinterpret_cast<double2*>(w),
                                                reinterpret_cast<double2*>(w), stream);
                    if (rc == SG_OK && hipStreamSynchronize(stream) != hipSuccess) rc = fail(SG_EHIP, "sync failed");
                }
            }
        }
        (void)hipFree(partial);
        (void)hipFree(coef);
        if (pin) (void)hipHostFree(pin);
        return rc;
    })
}

int sg_norm(long long n, const sg_c64* x, double* out_host, hipStream_t stream) {
    SG_TRY({
        if (n < 1 || !x || !out_host) return fail(SG_EINVAL, "invalid argument");
        const int nb = sgi::reduction_blocks(n);
        double2 *partial = nullptr, *coef = nullptr;
        int rc = SG_OK;
        if (hipMalloc(&partial, (size_t)nb * sizeof(double2)) != hipSuccess ||
            hipMalloc(&coef, sizeof(double2)) != hipSuccess) {
            rc = fail(SG_ENOMEM, "sg_norm scratch allocation failed");
        } else {
            rc = sgi::launch_norm2(n, reinterpret_cast<const double2*>(x), partial, nb, stream);
            if (rc == SG_OK) rc = sgi::launch_reduce_norm(nb, partial, coef, stream);
            double2 hv;
            if (rc == SG_OK && (hipMemcpyAsync(&hv, coef, sizeof(double2), hipMemcpyDeviceToHost, stream) != hipSuccess ||
                                hipStreamSynchronize(stream) != hipSuccess))
                rc = fail(SG_EHIP, "sg_norm copy failed");
            if (rc == SG_OK) *out_host = hv.x;
        }
        (void)hipFree(partial);
        (void)hipFree(coef);
        return rc;
    })
}

int sg_axpby(long long n, sg_c64 alpha, const sg_c64* x, sg_c64 beta, const sg_c64* y, sg_c64* out,
             hipStream_t stream) {
    SG_TRY({
        if (n < 1 || !x || !out) return fail(SG_EINVAL, "invalid argument");
        if (!y && (beta.re != 0.0 || beta.im != 0.0)) return fail(SG_EINVAL, "sg_axpby: y is NULL but beta is not 0");
        return sgi::launch_axpby(n, make_double2(alpha.re, alpha.im), reinterpret_cast<const double2*>(x),
                                 make_double2(beta.re, beta.im), reinterpret_cast<const double2*>(y),
                                 reinterpret_cast<double2*>(out), stream);
    })
}

int sg_gmres_batched(int count, const sg_handle* handles, const sg_c64* const* b, sg_c64* const* x,
                     const sg_solve_opts* opts, sg_solve_stats* stats, hipStream_t stream) {
    SG_TRY({
        if (count < 0) return fail(SG_EINVAL, "count must be >= 0");
        if (count == 0) return SG_OK;
        if (!handles || !b || !x || !opts) return fail(SG_EINVAL, "null argument");
        std::vector<Ctx*> cs(count);
        std::vector<const double2*> bs(count);
        std::vector<double2*> xs(count);
        for (int i = 0; i < count; ++i) {
            if (!handles[i]) return fail(SG_EINVAL, "null handle in the batch");
            cs[i] = ctx(handles[i]);
            if (int rc = guard_device(cs[i])) return rc;
            bs[i] = reinterpret_cast<const double2*>(b[i]);
            xs[i] = reinterpret_cast<double2*>(x[i]);
        }
        ProfBind pb(cs[0]);
        return sgi::run_gmres_batched(count, cs.data(), bs.data(), xs.data(), opts, stats, stream);
    })
}

int sg_batched_release(void) {
    SG_TRY({ return sgi::batched_release(); })
}

int sg_autotune(int count, const sg_handle* handles, int precision, int reps, double* ms_total, hipStream_t stream) {
    SG_TRY({
        if (count < 0 || (count > 0 && !handles)) return fail(SG_EINVAL, "invalid handle list");
        std::vector<Ctx*> cs(count);
        for (int i = 0; i < count; ++i) {
            if (!handles[i]) return fail(SG_EINVAL, "null handle");
            cs[i] = ctx(handles[i]);
            if (int rc = guard_device(cs[i])) return rc;
        }
        return sgi::autotune(count, cs.data(), precision, reps, ms_total, stream);
    })
}

int sg_tune_get(int n, int Q, int precision) {
    SG_TRY({ return sgi::tune_get(n, Q, precision); })
}

int sg_tune_set(int n, int Q, int precision, int tile) {
    SG_TRY({
        if (tile < 0 || tile >= sgi::SG_GEMM_NCFG) return fail(SG_EINVAL, "unknown tile shape");
        if (!sgi::gemm_cfg_valid(tile, precision)) return fail(SG_EINVAL, "tile shape not available in this precision");
        if (n < 1 || Q < 1 || precision < SG_PREC_F64 || precision > SG_PREC_BF16X3)
            return fail(SG_EINVAL, "invalid table key");
        sgi::tune_set(n, Q, precision, tile);
        return SG_OK;
    })
}

static sgi::Net* netp(sg_net n) { return reinterpret_cast<sgi::Net*>(n); }

static int guard_net(sgi::Net* n) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SG_EHIP, "hipGetDevice failed");
    if (dev != n->device) return fail(SG_EINVAL, "network was created on another device");
    return SG_OK;
}

int sg_net_create(int Q, int s, unsigned long long seed, sg_net* out) {
    SG_TRY({
        if (!out) return fail(SG_EINVAL, "out is null");
        *out = nullptr;
        sgi::Net* n = nullptr;
        int rc = sgi::net_create(Q, s, seed, &n);
        if (rc) return rc;
        *out = reinterpret_cast<sg_net>(n);
        return SG_OK;
    })
}

void sg_net_destroy(sg_net net) {
    try {
        delete netp(net);
    } catch (...) {
    }
}

long long sg_net_num_params(sg_net net) { return net ? netp(net)->nparams : 0; }

int sg_net_get_params(sg_net net, float* host) {
    SG_TRY({
        if (!net || !host) return fail(SG_EINVAL, "null argument");
        if (int rc = guard_net(netp(net))) return rc;
        return sgi::net_get_params(netp(net), host);
    })
}

int sg_net_set_params(sg_net net, const float* host) {
    SG_TRY({
        if (!net || !host) return fail(SG_EINVAL, "null argument");
        if (int rc = guard_net(netp(net))) return rc;
        return sgi::net_set_params(netp(net), host);
    })
}

int sg_net_forward_nhwc(sg_net net, int batch, int H, const float* x, float* y, hipStream_t stream) {
    SG_TRY({
        if (!net || !x || !y) return fail(SG_EINVAL, "null argument");
        if (int rc = guard_net(netp(net))) return rc;
        return sgi::net_forward_nhwc(netp(net), batch, H, x, y, stream);
    })
}

int sg_net_grad_nhwc(sg_net net, int batch, int H, const float* x, const float* t, double* loss, float* grad_host,
                     hipStream_t stream) {
    SG_TRY({
        if (!net || !x || !t) return fail(SG_EINVAL, "null argument");
        if (int rc = guard_net(netp(net))) return rc;
        return sgi::net_grad_nhwc(netp(net), batch, H, x, t, loss, grad_host, stream);
    })
}

int sg_net_adam_step(sg_net net, float lr, hipStream_t stream) {
    SG_TRY({
        if (!net || !(lr > 0)) return fail(SG_EINVAL, "invalid argument");
        if (int rc = guard_net(netp(net))) return rc;
        return sgi::net_adam_step(netp(net), lr, stream);
    })
}

int sg_net_train_pairs(sg_net net, int batch, const sg_handle* handles, const sg_c64* const* r, const sg_c64* const* e,
                       float lr, int precision, double* loss, hipStream_t stream) {
    SG_TRY({
        if (!net || !handles || !r || !e || batch < 1 || !(lr > 0)) return fail(SG_EINVAL, "invalid argument");
        if (precision < SG_PREC_F64 || precision > SG_PREC_BF16X3) return fail(SG_EINVAL, "unknown precision");
        if (int rc = guard_net(netp(net))) return rc;
        std::vector<Ctx*> cs(batch);
        std::vector<const double2*> rs(batch), es(batch);
        for (int i = 0; i < batch; ++i) {
            if (!handles[i]) return fail(SG_EINVAL, "null handle");
            cs[i] = ctx(handles[i]);
            rs[i] = reinterpret_cast<const double2*>(r[i]);
            es[i] = reinterpret_cast<const double2*>(e[i]);
        }
        return sgi::net_train_pairs(netp(net), batch, cs.data(), rs.data(), es.data(), lr, precision, loss, stream);
    })
}

int sg_net_save(sg_net net, const char* path) {
    SG_TRY({
        if (!net || !path) return fail(SG_EINVAL, "null argument");
        return sgi::net_save(netp(net), path);
    })
}

int sg_net_load(sg_net net, const char* path) {
    SG_TRY({
        if (!net || !path) return fail(SG_EINVAL, "null argument");
        return sgi::net_load(netp(net), path);
    })
}

int sg_attach_net(sg_handle h, sg_net net) {
    SG_TRY({
        if (!h) return fail(SG_EINVAL, "null handle");
        Ctx* c = ctx(h);
        if (net) {
            sgi::Net* n = netp(net);
            if (n->device != c->device) return fail(SG_EINVAL, "network and handle are on different devices");
            if (c->vmean) return fail(SG_EINVAL, "the learned correction needs a constant mean wavenumber solved by fast diagonalisation");
            if (c->dim != 2 || n->Q != c->Q || n->s != c->s)
                return fail(SG_EINVAL, "network shape does not match the problem (2D, same Q and s)");
        }
        c->net = netp(net);
        return SG_OK;
    })
}

int sg_set_profiling(sg_handle h, int on) {
    SG_TRY({
        if (!h) return fail(SG_EINVAL, "null handle");
        Ctx* c = ctx(h);
        c->prof.reset();
        c->prof.on = on != 0;
        c->prof.mask = ~0u;
        return SG_OK;
    })
}

int sg_profile_kinds(sg_handle h, unsigned mask) {
    SG_TRY({
        if (!h) return fail(SG_EINVAL, "null handle");
        ctx(h)->prof.mask = mask;
        return SG_OK;
    })
}

int sg_kernel_times(sg_handle h, int nkinds, double* ms, long long* count, double* work) {
    SG_TRY({
        if (!h || nkinds < 0) return fail(SG_EINVAL, "invalid argument");
        Ctx* c = ctx(h);
        if (int rc = c->prof.resolve()) return rc;
        for (int k = 0; k < nkinds; ++k) {
            const bool in = k < SG_K_NKINDS;
            if (ms) ms[k] = in ? c->prof.ms[k] : 0.0;
            if (count) count[k] = in ? c->prof.cnt[k] : 0;
            if (work) work[k] = in ? c->prof.work[k] : 0.0;
        }
        return SG_OK;
    })
}

const char* sg_strerror(int status) {
    switch (status) {
        case SG_OK: return "ok";
        case SG_ENOTCONV: return "not converged (maxit reached)";
        case SG_FALLBACK_USED: return "learned correction rejected, plain path used";
        case SG_EINVAL: return "invalid argument";
        case SG_ENOMEM: return "out of memory";
        case SG_EHIP: return "HIP runtime error";
        case SG_EBREAKDOWN: return "Krylov breakdown";
        case SG_ENONFINITE: return "non-finite value";
        case SG_ESETUP: return "setup validation failed";
        default: return "unknown status";
    }
}

const char* sg_last_error(void) { return sgi::last_error(); }

}  // extern "C"
