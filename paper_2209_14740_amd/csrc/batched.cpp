// Batched restarted GMRES over many independent SG systems of uneven size (grid N and
// PC size Q differ per instance), and the tile-shape autotuner of its GEMMs.
//
// Every instance runs the right-preconditioned GMRES(m) of dcgs2.cpp (the mean-value or
// mean-CSL block solve of Section 5, delayed-CGS2 Arnoldi in the flexible form, Givens
// least squares, FP64 true residual at the end of every cycle), or that of gmres.cpp
// (two-pass CGS2) when every handle asks for it.  The batch advances in lockstep steps: in one
// step each active instance does one unit of work (start, one Arnoldi step, or the end of
// a cycle), and every phase of the step is ONE grouped launch over all instances (the
// block → instance map is a prefix table), followed by one host synchronisation for the
// whole batch.  Instances wait in a queue sorted by estimated cost, largest first, and
// enter slots whose Krylov workspaces are carved from one device arena; a finished
// instance frees its slot for the next one in the queue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "apply_args.h"
#include "sg_internal.h"

namespace sgi {

// ---- autotuner table ------------------------------------------------------------------

namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tune;   // (n, Q, precision) → GEMM tile configuration
}  // namespace

int tune_get(int n, int Q, int precision) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find({n, Q, precision});
    return it == g_tune.end() ? -1 : it->second;
}

void tune_set(int n, int Q, int precision, int cfg) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[{n, Q, precision}] = cfg;
}

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// A grouped launch under construction: tasks and the prefix of their block counts.
template <class T>
struct Group {
    std::vector<T> tasks;
    std::vector<int> start{0};
    size_t off_tasks = 0, off_start = 0;   // byte offsets in the staging buffer
    double work = 0;
    int maxnv = 0;
    void add(const T& t, int blocks, double w = 0) {
        tasks.push_back(t);
        start.push_back(start.back() + blocks);
        work += w;
    }
    int n() const { return (int)tasks.size(); }
    int total() const { return start.back(); }
    void clear() {
        tasks.clear();
        start.assign(1, 0);
        work = 0;
        maxnv = 0;
    }
};

// Host-to-device staging of one step: all task tables, the lazy scales and the
// least-squares coefficients, uploaded with one copy.
struct Staging {
    std::vector<unsigned char> host;
    unsigned char* pinned = nullptr;
    unsigned char* dev = nullptr;
    size_t cap = 0;
    size_t used = 0;
    void reset() {
        host.clear();
        used = 0;
    }
    size_t put(const void* p, size_t bytes) {
        const size_t off = align_up(used);
        host.resize(off + bytes);
        if (bytes) std::memcpy(host.data() + off, p, bytes);
        used = off + bytes;
        return off;
    }
    template <class T>
    void put_group(Group<T>& g) {
        g.off_tasks = put(g.tasks.data(), g.tasks.size() * sizeof(T));
        g.off_start = put(g.start.data(), g.start.size() * sizeof(int));
    }
    template <class T>
    const T* dtasks(const Group<T>& g) const { return reinterpret_cast<const T*>(dev + g.off_tasks); }
    template <class T>
    const int* dstart(const Group<T>& g) const { return reinterpret_cast<const int*>(dev + g.off_start); }
    int ensure(size_t bytes) {
        if (bytes <= cap) return SG_OK;
        if (pinned) (void)hipHostFree(pinned);
        if (dev) (void)hipFree(dev);
        pinned = nullptr;
        dev = nullptr;
        cap = std::max(bytes, (size_t)1 << 20);
        SG_HIP(hipHostMalloc(&pinned, cap, hipHostMallocDefault));
        if (hipMalloc(&dev, cap) != hipSuccess) return fail(SG_ENOMEM, "batched solve: staging allocation failed");
        return SG_OK;
    }
    ~Staging() {
        if (pinned) (void)hipHostFree(pinned);
        if (dev) (void)hipFree(dev);
    }
};

constexpr int kMaxDev = 64;
struct ArenaCache {
    std::mutex mu;
    unsigned char* p = nullptr;
    size_t bytes = 0;
};
ArenaCache g_arena[kMaxDev];

// First-fit allocator over one device arena (offsets; freed ranges are merged).
struct Arena {
    unsigned char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset → length
    void init(unsigned char* b, size_t s) {
        base = b;
        size = s;
        free_.clear();
        free_[0] = s;
    }
    bool alloc(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

enum Phase { FREE = 0, INIT, ARN, END, DONE };

using cd = std::complex<double>;

struct Slot {
    int inst = -1;
    Ctx* c = nullptr;
    const double2* b = nullptr;
    double2* x = nullptr;
    double2* V = nullptr;      // (m+1) vectors
    double2* zt = nullptr;     // preconditioned vector
    double2* ut = nullptr;     // scratch vector
    double2* partial = nullptr;
    int nblk = 0;
    size_t off = 0, bytes = 0;
    int phase = FREE;
    int j = 0, k = 0;
    bool breakdown = false;
    double bnorm = 0;
    std::vector<cd> H, R, g, sn, y;
    std::vector<double> cs, hscale;
    sg_solve_stats st{};
    std::chrono::steady_clock::time_point t0;
};

double cost_estimate(const Ctx* c) {
    const double n = c->n, P = (double)c->P, Q = c->Q;
    return Q * (c->dim == 2 ? 16.0 * n * n * n / 100.0 : 0.0) + Q * P * 40.0;
}

}  // namespace

// ---- delayed-CGS2 form ---------------------------------------------------------------------
//
// The per-instance process of dcgs2.cpp in lockstep steps: the Arnoldi process in the
// flexible form (z_j = P^{-1} u_j kept in a Z basis, x += Z y), the second Gram-Schmidt pass
// delayed by one step, so that each step reads an instance's basis twice (one reduction,
// one update) instead of three times.  Column j-1 of H is complete at step j; when the
// predicted residual of column j reaches the tolerance (or the cycle is full) step j+1 is a
// finishing reduction of u_{j+1} alone.  The first step of an instance also copies b into
// the basis and zeroes x; a cycle end forms x += Z y and the true residual r = b - A x in
// slot 0, the next cycle's candidate u_0.
namespace {

struct DSlot {
    int inst = -1;
    Ctx* c = nullptr;
    const double2* b = nullptr;
    double2* x = nullptr;
    double2 *V = nullptr, *Z = nullptr, *ut = nullptr, *partial = nullptr;
    double2 *red = nullptr, *h1 = nullptr, *cv = nullptr, *cw = nullptr, *cu = nullptr;
    int nblk = 0;
    size_t off = 0, bytes = 0;
    bool used = false;
    bool start = false;     // the next step also copies b into slot 0 and zeroes x
    bool end = false;       // the next step is a cycle end (x += Z y, residual)
    bool full = true;       // the next Arnoldi step is a full one (else a finishing reduction)
    bool breakdown = false;
    int j = 0, k = 0;
    double bnorm = 0, est = 1.0;
    std::vector<cd> R, g, sn, y;
    std::vector<double> cs;
    sg_solve_stats st{};
    std::chrono::steady_clock::time_point t0;

    void new_cycle(int m) {
        R.assign((size_t)(m + 1) * m, 0.0);
        g.assign(m + 1, 0.0);
        sn.assign(m, 0.0);
        cs.assign(m, 0.0);
        j = 0;
        k = 0;
        full = true;
        end = false;
    }
    // Givens rotation of column jj (entries col[0..jj+1]); returns |g_{jj+1}|.  Without
    // commit nothing is stored (a prediction).
    double add(int m, int jj, std::vector<cd> col, bool commit) {
        for (int i = 0; i < jj; ++i) {
            const cd t = cs[i] * col[i] + sn[i] * col[i + 1];
            col[i + 1] = -std::conj(sn[i]) * col[i] + cs[i] * col[i + 1];
            col[i] = t;
        }
        const cd a = col[jj], bb = col[jj + 1];
        double cj;
        cd sj;
        if (std::abs(bb) == 0.0) { cj = 1.0; sj = 0.0; }
        else if (std::abs(a) == 0.0) { cj = 0.0; sj = std::conj(bb) / std::abs(bb); }
        else {
            const double t = std::hypot(std::abs(a), std::abs(bb));
            cj = std::abs(a) / t;
            sj = (a / std::abs(a)) * std::conj(bb) / t;
        }
        const cd gnext = -std::conj(sj) * g[jj];
        if (commit) {
            cs[jj] = cj;
            sn[jj] = sj;
            col[jj] = cj * a + sj * bb;
            col[jj + 1] = 0.0;
            for (int i = 0; i <= jj + 1; ++i) R[(size_t)i * m + jj] = col[i];
            g[jj + 1] = gnext;
            g[jj] = cj * g[jj];
        }
        return std::abs(gnext);
    }
};

}  // namespace

static int run_gmres_batched_dcgs(int count, Ctx* const* ctx, const double2* const* b, double2* const* x,
                                  const sg_solve_opts* o, sg_solve_stats* stats, hipStream_t stream) {
    const int m = o->restart;
    const int pc = o->precond, prec = o->precision;
    const int RW = 2 * m + 3;        // record words per slot (also holds a cycle end's residual norm)
    const int SW = 6 * m + 16;       // small device words per slot: red, h1, cv, cw, cu (7)
    std::vector<size_t> need(count);
    size_t largest = 0, total = 0;
    for (int i = 0; i < count; ++i) {
        const size_t nv = (size_t)ctx[i]->nvec;
        need[i] = align_up((size_t)(2 * m + 2) * nv * sizeof(double2)) +
                  align_up((size_t)reduction_blocks(ctx[i]->nvec) * RW * sizeof(double2)) +
                  align_up((size_t)SW * sizeof(double2));
        largest = std::max(largest, need[i]);
        total += need[i];
    }
    int dev = 0;
    SG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) return fail(SG_EINVAL, "batched solve: device index out of range");
    ArenaCache& ac = g_arena[dev];
    std::lock_guard<std::mutex> arena_lock(ac.mu);
    size_t freeb = 0, totb = 0;
    SG_HIP(hipMemGetInfo(&freeb, &totb));
    const size_t avail = freeb + ac.bytes;
    const size_t arena_bytes = std::min(total, std::max(largest, avail / 2));
    if (arena_bytes > avail) return fail(SG_ENOMEM, "batched solve: not enough device memory for one instance");
    if (ac.bytes < arena_bytes) {
        SG_HIP(hipStreamSynchronize(stream));
        (void)hipFree(ac.p);
        ac.p = nullptr;
        ac.bytes = 0;
        if (hipMalloc(&ac.p, arena_bytes) != hipSuccess) return fail(SG_ENOMEM, "batched solve: arena allocation failed");
        ac.bytes = arena_bytes;
    }
    Arena arena;
    arena.init(ac.p, arena_bytes);

    std::vector<int> queue(count);
    for (int i = 0; i < count; ++i) queue[i] = i;
    std::stable_sort(queue.begin(), queue.end(),
                     [&](int a, int c2) { return cost_estimate(ctx[a]) > cost_estimate(ctx[c2]); });
    size_t qhead = 0;

    const int S = count;
    std::vector<DSlot> slots(S);
    double2* d_rec = nullptr;
    if (hipMalloc(&d_rec, (size_t)S * RW * sizeof(double2)) != hipSuccess)
        return fail(SG_ENOMEM, "batched solve: record table allocation failed");
    struct FreeD {
        double2* p;
        ~FreeD() { (void)hipFree(p); }
    } free_rec{d_rec};
    double2* h_rec = nullptr;
    SG_HIP(hipHostMalloc(&h_rec, (size_t)S * RW * sizeof(double2), hipHostMallocDefault));
    struct FreeH {
        double2* p;
        ~FreeH() { (void)hipHostFree(p); }
    } free_hrec{h_rec};
    int tri_nr = 2;
    if (pc == SG_PC_NONE) tri_nr = 1;
    for (int i = 0; i < count && tri_nr == 2; ++i)
        if (!tri_nr_ok(ctx[i]->tri[pc == SG_PC_MEAN ? 0 : 1], ctx[i]->n, ctx[i]->Q, ctx[i]->dim)) tri_nr = 1;
    // the reduced-precision forms keep the 2D transform intermediate in FP32, as sg_precond does
    const bool t32 = prec != SG_PREC_F64;
    int tri_nr32 = pc == SG_PC_NONE ? 1 : 2;
    for (int i = 0; i < count && tri_nr32 == 2; ++i)
        if (ctx[i]->dim == 2 && !tri_nr_ok32(ctx[i]->tri[pc == SG_PC_MEAN ? 0 : 1], ctx[i]->n, ctx[i]->Q, 2))
            tri_nr32 = 1;
    hipEvent_t step_done = nullptr;
    SG_HIP(hipEventCreateWithFlags(&step_done, hipEventDisableTiming));
    struct FreeE {
        hipEvent_t e;
        ~FreeE() { (void)hipEventDestroy(e); }
    } free_ev{step_done};
    Staging stg;

    std::vector<int> active;
    bool any_notconv = false;
    Group<VecTask> g_copy, g_lin, g_pcopy, g_xupd, g_res, g_norm, g_nred;
    Group<ApplyArgs> g_apply;
    std::map<std::pair<int, int>, Group<ApplyArgs>> g_spec;
    Group<TriTask> g_tri, g_tri32;
    std::vector<Group<GemmTask>> g_fwd(SG_GEMM_NCFG), g_inv(SG_GEMM_NCFG);
    Group<DcgsTask> g_dred, g_dsum, g_dfin, g_dupd;
    std::vector<double2> y_tab((size_t)S * (m + 1));

    auto admit = [&]() {
        while (qhead < queue.size()) {
            const int i = queue[qhead];
            size_t off = 0;
            if (!arena.alloc(need[i], &off)) break;
            int sidx = -1;
            for (int sI = 0; sI < S; ++sI)
                if (!slots[sI].used) { sidx = sI; break; }
            if (sidx < 0) { arena.release(off, need[i]); break; }
            ++qhead;
            DSlot& s = slots[sidx];
            s = DSlot{};
            s.used = true;
            s.inst = i;
            s.c = ctx[i];
            s.b = b[i];
            s.x = x[i];
            s.off = off;
            s.bytes = need[i];
            const size_t nv = (size_t)s.c->nvec;
            unsigned char* p = arena.base + off;
            s.V = reinterpret_cast<double2*>(p);
            s.Z = s.V + (size_t)(m + 1) * nv;
            s.ut = s.Z + (size_t)m * nv;
            p += align_up((size_t)(2 * m + 2) * nv * sizeof(double2));
            s.partial = reinterpret_cast<double2*>(p);
            s.nblk = reduction_blocks(s.c->nvec);
            p += align_up((size_t)s.nblk * RW * sizeof(double2));
            s.red = reinterpret_cast<double2*>(p);   // 2m+3
            s.h1 = s.red + RW;                       // m+1
            s.cv = s.h1 + (m + 1);                   // m
            s.cw = s.cv + m;                         // m
            s.cu = s.cw + m;                         // 7
            s.new_cycle(m);
            s.start = true;
            s.st.t_setup = s.c->t_setup_ms;
            s.t0 = std::chrono::steady_clock::now();
            active.push_back(sidx);
        }
    };
    auto vt_base = [&](const DSlot& s) {
        VecTask t{};
        t.n = s.c->nvec;
        t.nblocks = s.nblk;
        t.ldv = s.c->nvec;
        return t;
    };

    admit();
    if (active.empty()) return fail(SG_ENOMEM, "batched solve: no instance fits the arena");
    int rc = SG_OK;
    while (!active.empty()) {
        for (auto* gp : {&g_copy, &g_lin, &g_pcopy, &g_xupd, &g_res, &g_norm, &g_nred}) gp->clear();
        g_apply.clear();
        for (auto& kv : g_spec) kv.second.clear();
        g_tri.clear();
        g_tri32.clear();
        for (auto& gg : g_fwd) gg.clear();
        for (auto& gg : g_inv) gg.clear();
        for (auto* gp : {&g_dred, &g_dsum, &g_dfin, &g_dupd}) gp->clear();
        stg.reset();
        int nslot = 0;
        for (int sI : active) nslot = std::max(nslot, sI + 1);
        for (int sI : active) {
            const DSlot& s = slots[sI];
            if (s.end)
                for (int i = 0; i < s.k; ++i) y_tab[(size_t)sI * (m + 1) + i] = make_double2(s.y[i].real(), s.y[i].imag());
        }
        const size_t off_y = stg.put(y_tab.data(), (size_t)nslot * (m + 1) * sizeof(double2));
        auto dy = [&](int sI) { return reinterpret_cast<const double2*>(stg.dev + off_y) + (size_t)sI * (m + 1); };
        {
            const size_t per = sizeof(VecTask) * 8 + sizeof(ApplyArgs) + sizeof(TriTask) + 2 * sizeof(GemmTask) +
                               4 * sizeof(DcgsTask) + 48 * 4;
            if ((rc = stg.ensure(align_up(stg.used) + (size_t)active.size() * per + 160 * ALIGN * 2))) return rc;
        }
        unsigned char* const dev_before = stg.dev;

        size_t lds = 0;
        auto add_apply = [&](Ctx* c, const double2* xin, double2* yout) {
            const ApplyArgs aa = make_apply_args(c, xin, yout);
            const double abytes = (double)c->P * (32.0 * c->Q + 8.0 * c->K.nfield);
            if (c->dim == 2 && c->use_spec_apply && c->op_csl_beta == 0.0 &&
                (long long)c->n * c->n * 16 < (1ll << 32) &&
                dispatch_spec_grouped(c->s, c->degree, nullptr, nullptr, 0, 0, nullptr)) {
                g_spec[{c->s, c->degree}].add(aa, spec_row_blocks(c->n), abytes);
            } else {
                g_apply.add(aa, aa.ntiles_x * aa.nrows, abytes);
                lds = std::max(lds, apply_lds_bytes(c->Q, c->K.nfield));
            }
        };
        int maxj = 0;
        for (int sI : active) {
            DSlot& s = slots[sI];
            Ctx* c = s.c;
            const long long n = c->nvec;
            double2* rec = d_rec + (size_t)sI * RW;
            if (s.end) {
                // x += Z y; r = b - A x into slot 0; ||r|| into the record
                VecTask t = vt_base(s);
                t.V = s.Z;
                t.nv = s.k;
                t.coef = dy(sI);
                t.w = s.ut;
                g_lin.add(t, s.nblk, 16.0 * (s.k + 1) * n);
                g_lin.maxnv = std::max(g_lin.maxnv, s.k);
                VecTask xu = vt_base(s);
                xu.x = s.x;
                xu.y = s.ut;
                xu.a = make_double2(1, 0);
                xu.b = make_double2(1, 0);
                xu.w = s.x;
                g_xupd.add(xu, s.nblk, 48.0 * n);
                add_apply(c, s.x, s.ut);
                VecTask r = vt_base(s);
                r.x = s.b;
                r.y = s.ut;
                r.a = make_double2(1, 0);
                r.b = make_double2(-1, 0);
                r.w = s.V;
                g_res.add(r, s.nblk, 48.0 * n);
                VecTask nm = vt_base(s);
                nm.V = s.V;
                nm.nv = 0;
                nm.w = s.V;
                nm.partial = s.partial;
                g_norm.add(nm, s.nblk, 16.0 * n);
                VecTask rn = nm;
                rn.out = rec;
                g_nred.add(rn, 1);
                continue;
            }
            if (s.start) {
                VecTask t = vt_base(s);   // u_0 = b (x = 0)
                t.x = s.b;
                t.a = make_double2(1, 0);
                t.w = s.V;
                g_copy.add(t, s.nblk, 32.0 * n);
                VecTask z = vt_base(s);
                z.a = make_double2(1, 0);
                z.w = s.x;
                g_copy.add(z, s.nblk, 16.0 * n);
            }
            const int j = s.j;
            double2* uj = s.V + (size_t)j * n;
            if (s.full) {
                double2* zj = s.Z + (size_t)j * n;
                if (pc == SG_PC_NONE || c->dim == 1) {
                    VecTask t = vt_base(s);
                    t.x = uj;
                    t.a = make_double2(1, 0);
                    t.w = zj;
                    g_pcopy.add(t, s.nblk, 32.0 * n);
                }
                if (pc != SG_PC_NONE) {
                    const TriFactors& f = c->tri[pc == SG_PC_MEAN ? 0 : 1];
                    if (c->dim == 1) {
                        TriTask tt = make_tri_task(f, zj, c->n, c->n, c->Q, 1, tri_nr);
                        g_tri.add(tt, tt.nblocks, 32.0 * n + 65.0 * f.nsys * c->n);
                    } else {
                        const int cfg = gemm_cfg_for(c->n, c->Q * c->n, prec);
                        const int M = c->Q * c->n;
                        GemmTask gf = make_gemm_task(prec, reinterpret_cast<const double*>(uj), c->n, c->fwd, c->n,
                                                     reinterpret_cast<double*>(c->d_tmp_pc), c->tld, M, cfg);
                        GemmTask gi = make_gemm_task(prec, reinterpret_cast<const double*>(c->d_tmp_pc), c->tld, c->inv,
                                                     c->n, reinterpret_cast<double*>(zj), c->n, M, cfg);
                        gf.io = t32 ? GEMM_IO_C32 : GEMM_IO_F64;
                        gi.io = t32 ? GEMM_IO_A32 : GEMM_IO_F64;
                        const double fl = (gemm_cfg_3m(cfg) ? 6.0 : 8.0) * M * (double)c->n * c->n;
                        g_fwd[cfg].add(gf, gf.tiles_m * gf.tiles_n, fl);
                        g_inv[cfg].add(gi, gi.tiles_m * gi.tiles_n, fl);
                        TriTask tt = make_tri_task(f, c->d_tmp_pc, c->n, c->tld, c->Q, 2, t32 ? tri_nr32 : tri_nr);
                        (t32 ? g_tri32 : g_tri).add(tt, tt.nblocks, (t32 ? 16.0 : 32.0) * n + 65.0 * f.nsys * c->n);
                    }
                }
                add_apply(c, zj, uj + n);
            }
            DcgsTask d{};
            d.V = s.V;
            d.ldv = n;
            d.n = n;
            d.partial = s.partial;
            d.red = s.red;
            d.h1 = s.h1;
            d.rec = rec;
            d.cv = s.cv;
            d.cw = s.cw;
            d.cu = s.cu;
            d.j = j;
            d.full = s.full ? 1 : 0;
            // about 32 grid-stride chunks of 64 elements per block (the launch holds every
            // instance's blocks, so the grid is full without short blocks), and from two basis
            // vectors per wave on at most 512 blocks per instance, as in the single solver
            d.nblocks = (int)std::min<long long>((j + 3) / 4 >= 2 ? 512 : s.nblk,
                                                 std::max<long long>(1, (n + 2047) / 2048));
            maxj = std::max(maxj, j);
            g_dred.add(d, d.nblocks, 16.0 * (j + (s.full ? 2 : 1)) * n);
            g_dsum.add(d, s.full ? 2 * j + 3 : j + 1);
            g_dfin.add(d, 1);
            if (s.full) g_dupd.add(d, d.nblocks, 16.0 * (j + 4) * n);
        }

        for (auto* gp : {&g_copy, &g_lin, &g_pcopy, &g_xupd, &g_res, &g_norm, &g_nred}) stg.put_group(*gp);
        stg.put_group(g_apply);
        for (auto& kv : g_spec) stg.put_group(kv.second);
        stg.put_group(g_tri);
        stg.put_group(g_tri32);
        for (auto& gg : g_fwd) stg.put_group(gg);
        for (auto& gg : g_inv) stg.put_group(gg);
        for (auto* gp : {&g_dred, &g_dsum, &g_dfin, &g_dupd}) stg.put_group(*gp);
        if (stg.used > stg.cap || stg.dev != dev_before) return fail(SG_EINVAL, "batched solve: staging overflow");
        std::memcpy(stg.pinned, stg.host.data(), stg.used);
        SG_HIP(hipMemcpyAsync(stg.dev, stg.pinned, stg.used, hipMemcpyHostToDevice, stream));

        // launches, in dependency order
        if ((rc = launch_axpby_grouped(stg.dtasks(g_copy), stg.dstart(g_copy), g_copy.n(), g_copy.total(), g_copy.work,
                                       stream)))
            return rc;
        if ((rc = launch_lincomb_grouped(stg.dtasks(g_lin), stg.dstart(g_lin), g_lin.n(), g_lin.total(), g_lin.maxnv,
                                         g_lin.work, stream)))
            return rc;
        if ((rc = launch_axpby_grouped(stg.dtasks(g_pcopy), stg.dstart(g_pcopy), g_pcopy.n(), g_pcopy.total(),
                                       g_pcopy.work, stream)))
            return rc;
        for (int cfg = 0; cfg < SG_GEMM_NCFG; ++cfg)
            if ((rc = launch_gemm_grouped(prec, cfg, t32 ? GEMM_IO_C32 : GEMM_IO_F64, stg.dtasks(g_fwd[cfg]),
                                          stg.dstart(g_fwd[cfg]), g_fwd[cfg].n(), g_fwd[cfg].total(), g_fwd[cfg].work,
                                          stream)))
                return rc;
        int max_seg = 0, max_seg32 = 0;
        for (const TriTask& tt : g_tri.tasks) max_seg = std::max(max_seg, tt.f.L);
        for (const TriTask& tt : g_tri32.tasks) max_seg32 = std::max(max_seg32, tt.f.L);
        if ((rc = launch_tri_grouped(stg.dtasks(g_tri), stg.dstart(g_tri), g_tri.n(), g_tri.total(), max_seg, tri_nr,
                                     false, g_tri.work, stream)))
            return rc;
        if ((rc = launch_tri_grouped(stg.dtasks(g_tri32), stg.dstart(g_tri32), g_tri32.n(), g_tri32.total(), max_seg32,
                                     tri_nr32, true, g_tri32.work, stream)))
            return rc;
        for (int cfg = 0; cfg < SG_GEMM_NCFG; ++cfg)
            if ((rc = launch_gemm_grouped(prec, cfg, t32 ? GEMM_IO_A32 : GEMM_IO_F64, stg.dtasks(g_inv[cfg]),
                                          stg.dstart(g_inv[cfg]), g_inv[cfg].n(), g_inv[cfg].total(), g_inv[cfg].work,
                                          stream)))
                return rc;
        if ((rc = launch_axpby_grouped(stg.dtasks(g_xupd), stg.dstart(g_xupd), g_xupd.n(), g_xupd.total(), g_xupd.work,
                                       stream)))
            return rc;
        if ((rc = launch_apply_grouped(stg.dtasks(g_apply), stg.dstart(g_apply), g_apply.n(), g_apply.total(), lds,
                                       g_apply.work, stream)))
            return rc;
        for (auto& kv : g_spec) {
            Group<ApplyArgs>& gg = kv.second;
            if (gg.n() == 0) continue;
            KScope ks(SG_K_APPLY, gg.work, stream);
            dispatch_spec_grouped(kv.first.first, kv.first.second, stg.dtasks(gg), stg.dstart(gg), gg.n(), gg.total(),
                                  stream);
            SG_HIP(hipGetLastError());
        }
        if ((rc = launch_axpby_grouped(stg.dtasks(g_res), stg.dstart(g_res), g_res.n(), g_res.total(), g_res.work,
                                       stream)))
            return rc;
        if ((rc = launch_dcgs_reduce_grouped(stg.dtasks(g_dred), stg.dstart(g_dred), g_dred.n(), g_dred.total(), maxj,
                                             g_dred.work, stream)))
            return rc;
        if ((rc = launch_dcgs_sum_grouped(stg.dtasks(g_dsum), stg.dstart(g_dsum), g_dsum.n(), g_dsum.total(), stream)))
            return rc;
        if ((rc = launch_dcgs_finalize_grouped(stg.dtasks(g_dfin), g_dfin.n(), stream))) return rc;
        if ((rc = launch_dcgs_update_grouped(stg.dtasks(g_dupd), stg.dstart(g_dupd), g_dupd.n(), g_dupd.total(), maxj,
                                             g_dupd.work, stream)))
            return rc;
        if ((rc = launch_upd_grouped(stg.dtasks(g_norm), stg.dstart(g_norm), g_norm.n(), g_norm.total(), 0, false,
                                     g_norm.work, stream)))
            return rc;
        if ((rc = launch_reduce_grouped(stg.dtasks(g_nred), stg.dstart(g_nred), g_nred.n(), g_nred.total(), 1, stream)))
            return rc;
        SG_HIP(hipMemcpyAsync(h_rec, d_rec, (size_t)nslot * RW * sizeof(double2), hipMemcpyDeviceToHost, stream));
        if ((rc = wait_stream(stream, step_done))) return rc;

        // host part of every active instance
        std::vector<int> still;
        for (int sI : active) {
            DSlot& s = slots[sI];
            const double2* hr = h_rec + (size_t)sI * RW;
            bool finished = false;
            if (s.end) {
                const double beta = hr[0].x;
                ++s.st.restarts;
                s.st.relres_true = beta / s.bnorm;
                if (!std::isfinite(beta)) {
                    s.st.relres_true = NAN;
                    finished = true;
                } else if (s.st.relres_true <= o->tol) {
                    s.st.converged = 1;
                    finished = true;
                } else if (s.breakdown || s.st.iters >= o->maxit) {
                    finished = true;
                } else {
                    s.new_cycle(m);   // u_0 = r is in slot 0
                    s.est = s.st.relres_true;
                }
            } else {
                const int j = s.j;
                const bool was_full = s.full;
                s.start = false;
                const double nu = hr[j].x;
                bool end = false;
                if (!std::isfinite(nu)) {
                    s.st.relres_true = NAN;
                    finished = true;
                } else if (j == 0) {
                    if (s.bnorm == 0.0) {   // first step of the solve: ||u_0|| = ||b||
                        s.bnorm = nu;
                        s.st.relres_true = 1.0;
                        if (nu == 0.0) {
                            s.st.converged = 1;
                            s.st.relres_true = 0.0;
                            finished = true;
                        }
                    }
                    s.g[0] = nu;
                } else if (s.k < j) {
                    // column j-1: rows 0..j-1 from the record, row j = ν_j
                    std::vector<cd> col(j + 1);
                    double colnorm = 0.0;
                    bool bad = false;
                    for (int i = 0; i < j; ++i) {
                        col[i] = cd(hr[i].x, hr[i].y);
                        if (!std::isfinite(col[i].real()) || !std::isfinite(col[i].imag())) bad = true;
                        colnorm += std::norm(col[i]);
                    }
                    col[j] = nu;
                    colnorm = std::sqrt(colnorm + nu * nu);
                    if (bad) {
                        s.st.relres_true = NAN;
                        finished = true;
                    } else {
                        const double gn = s.add(m, j - 1, col, true);
                        ++s.st.iters;
                        s.k = j;
                        s.est = gn / s.bnorm;
                        s.st.relres_est = s.est;
                        s.breakdown = !(nu > 1e-14 * colnorm);
                        end = s.breakdown || s.est <= o->tol || s.st.iters >= o->maxit || j == m;
                    }
                }
                if (!finished && end) {
                    const int k = s.k;
                    s.y.assign(k, 0.0);
                    bool bad = false;
                    for (int i = k - 1; i >= 0; --i) {
                        cd acc = s.g[i];
                        for (int l = i + 1; l < k; ++l) acc -= s.R[(size_t)i * m + l] * s.y[l];
                        s.y[i] = acc / s.R[(size_t)i * m + i];
                        if (!std::isfinite(s.y[i].real()) || !std::isfinite(s.y[i].imag())) bad = true;
                    }
                    if (bad) {
                        s.st.relres_true = NAN;
                        finished = true;
                    } else {
                        s.end = true;
                    }
                } else if (!finished && !was_full) {
                    s.full = true;   // the finishing reduction fell short: step j again, in full
                } else if (!finished) {
                    // predict column j from step j's record: first-pass projection of w_j and
                    // ||u_{j+1}||² = ||w_j||² - ||h||²; decide the kind of step j+1
                    const double pred = hr[2 * j + 2].y;
                    std::vector<cd> pcol(j + 2);
                    for (int i = 0; i <= j; ++i) pcol[i] = cd(hr[j + 1 + i].x, hr[j + 1 + i].y);
                    pcol[j + 1] = pred > 0.0 ? std::sqrt(pred) : 0.0;
                    const double pest = s.add(m, j, pcol, false) / s.bnorm;
                    const bool finish_next = j + 1 == m || s.st.iters + 1 >= o->maxit ||
                                             (s.est <= 30.0 * o->tol && pest <= o->tol);
                    s.j = j + 1;
                    s.full = !finish_next;
                }
            }
            if (finished) {
                s.st.t_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - s.t0).count();
                if (!s.st.converged) any_notconv = true;
                if (stats) stats[s.inst] = s.st;
                arena.release(s.off, s.bytes);
                s.used = false;
            } else {
                still.push_back(sI);
            }
        }
        active.swap(still);
        admit();
        if (active.empty() && qhead < queue.size()) return fail(SG_ENOMEM, "batched solve: arena fragmentation");
    }
    return any_notconv ? SG_ENOTCONV : SG_OK;
}

int run_gmres_batched(int count, Ctx* const* ctx, const double2* const* b, double2* const* x,
                      const sg_solve_opts* o, sg_solve_stats* stats, hipStream_t stream) {
    if (count < 0) return fail(SG_EINVAL, "count must be >= 0");
    if (count == 0) return SG_OK;
    if (!ctx || !b || !x || !o) return fail(SG_EINVAL, "null argument");
    if (o->restart < 1 || o->restart > 63) return fail(SG_EINVAL, "batched restart must be in [1, 63]");
    if (o->maxit < 1) return fail(SG_EINVAL, "maxit must be >= 1");
    if (!(o->tol > 0)) return fail(SG_EINVAL, "tol must be positive");
    if (o->precond < SG_PC_NONE || o->precond > SG_PC_CSL_MEAN) return fail(SG_EINVAL, "unsupported preconditioner");
    if (o->precision < SG_PREC_F64 || o->precision > SG_PREC_BF16X3) return fail(SG_EINVAL, "unknown precision");
    if (o->side != 0) return fail(SG_EINVAL, "batched solve: right preconditioning only");
    for (int i = 0; i < count; ++i)
        if (ctx[i] && ctx[i]->vmean)
            return fail(SG_EINVAL, "batched solve: handles whose mean block is solved by the line factorisation (spatially varying mean, or the eigenfactor fallback) are not supported");
    const int m = o->restart;
    const int pc = o->precond, prec = o->precision;

    // per-instance workspace: (m+1) basis vectors, zt, ut, reduction partials
    std::vector<size_t> need(count);
    size_t largest = 0, total = 0;
    for (int i = 0; i < count; ++i) {
        if (!ctx[i] || !b[i] || !x[i]) return fail(SG_EINVAL, "null handle or vector in the batch");
        if (b[i] == x[i]) return fail(SG_EINVAL, "b and x must not alias");
        for (int l = 0; l < i; ++l)
            if (ctx[l] == ctx[i]) return fail(SG_EINVAL, "a handle appears twice in the batch");
        const size_t nv = (size_t)ctx[i]->nvec;
        need[i] = align_up((size_t)(m + 3) * nv * sizeof(double2)) +
                  align_up((size_t)reduction_blocks(ctx[i]->nvec) * (m + 2) * sizeof(double2));
        largest = std::max(largest, need[i]);
        total += need[i];
    }
    // the delayed-CGS2 form unless a handle asks for the two-pass CGS2 (sg_set_orthogonalisation)
    bool dcgs = true;
    for (int i = 0; i < count; ++i) dcgs = dcgs && !ctx[i]->classic_cgs2;
    if (dcgs) return run_gmres_batched_dcgs(count, ctx, b, x, o, stats, stream);
    // The arena is kept per device between calls (a fresh allocation of this size costs far
    // more than the solves: the driver clears the memory it hands out); calls on one device
    // are serialised by its lock.
    int dev = 0;
    SG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) return fail(SG_EINVAL, "batched solve: device index out of range");
    ArenaCache& ac = g_arena[dev];
    std::lock_guard<std::mutex> arena_lock(ac.mu);
    size_t freeb = 0, totb = 0;
    SG_HIP(hipMemGetInfo(&freeb, &totb));
    const size_t avail = freeb + ac.bytes;   // the cached arena counts as available
    size_t arena_bytes = std::min(total, std::max(largest, avail / 2));
    if (arena_bytes > avail) return fail(SG_ENOMEM, "batched solve: not enough device memory for one instance");
    if (ac.bytes < arena_bytes) {
        SG_HIP(hipStreamSynchronize(stream));   // the previous call's work on the arena has ended
        (void)hipFree(ac.p);
        ac.p = nullptr;
        ac.bytes = 0;
        if (hipMalloc(&ac.p, arena_bytes) != hipSuccess) return fail(SG_ENOMEM, "batched solve: arena allocation failed");
        ac.bytes = arena_bytes;
    }
    unsigned char* arena_mem = ac.p;
    Arena arena;
    arena.init(arena_mem, arena_bytes);

    // queue: largest estimated cost first
    std::vector<int> queue(count);
    for (int i = 0; i < count; ++i) queue[i] = i;
    std::stable_sort(queue.begin(), queue.end(),
                     [&](int a, int c2) { return cost_estimate(ctx[a]) > cost_estimate(ctx[c2]); });
    size_t qhead = 0;

    const int S = count;   // at most one slot per instance
    std::vector<Slot> slots(S);
    const int CW = 3 * (m + 2);   // coefficient words per slot
    double2* d_coef = nullptr;
    if (hipMalloc(&d_coef, (size_t)S * CW * sizeof(double2)) != hipSuccess)
        return fail(SG_ENOMEM, "batched solve: coefficient table allocation failed");
    struct FreeC {
        double2* p;
        ~FreeC() { (void)hipFree(p); }
    } free_coef{d_coef};
    double2* h_coef = nullptr;
    SG_HIP(hipHostMalloc(&h_coef, (size_t)S * CW * sizeof(double2), hipHostMallocDefault));
    struct FreeH {
        double2* p;
        ~FreeH() { (void)hipHostFree(p); }
    } free_hcoef{h_coef};
    // sweep layout of every grouped launch: two right-hand sides per thread when all
    // instances allow it
    int tri_nr = 2;
    if (pc == SG_PC_NONE) tri_nr = 1;
    for (int i = 0; i < count && tri_nr == 2; ++i)
        if (!tri_nr_ok(ctx[i]->tri[pc == SG_PC_MEAN ? 0 : 1], ctx[i]->n, ctx[i]->Q, ctx[i]->dim)) tri_nr = 1;
    // the reduced-precision forms keep the 2D transform intermediate in FP32, as sg_precond does
    const bool t32 = prec != SG_PREC_F64;
    int tri_nr32 = pc == SG_PC_NONE ? 1 : 2;
    for (int i = 0; i < count && tri_nr32 == 2; ++i)
        if (ctx[i]->dim == 2 && !tri_nr_ok32(ctx[i]->tri[pc == SG_PC_MEAN ? 0 : 1], ctx[i]->n, ctx[i]->Q, 2))
            tri_nr32 = 1;
    hipEvent_t step_done = nullptr;   // the host polls it at the end of every lockstep step
    SG_HIP(hipEventCreateWithFlags(&step_done, hipEventDisableTiming));
    struct FreeE {
        hipEvent_t e;
        ~FreeE() { (void)hipEventDestroy(e); }
    } free_ev{step_done};
    Staging stg;

    std::vector<int> active;
    int ndone = 0;
    bool any_notconv = false;

    Group<VecTask> g_copy, g_lin, g_xupd, g_res, g_mdot, g_red1, g_upd1, g_red2, g_updn, g_redn, g_pcopy;
    Group<ApplyArgs> g_apply;                                  // generic operator
    std::map<std::pair<int, int>, Group<ApplyArgs>> g_spec;   // shape-specialised operator per (s, r)
    Group<TriTask> g_tri, g_tri32;
    std::vector<Group<GemmTask>> g_fwd(SG_GEMM_NCFG), g_inv(SG_GEMM_NCFG);
    std::vector<double> hscale_tab((size_t)S * (m + 2), 1.0);
    std::vector<double2> y_tab((size_t)S * (m + 1));

    auto admit = [&]() -> int {
        while (qhead < queue.size()) {
            const int i = queue[qhead];
            size_t off = 0;
            if (!arena.alloc(need[i], &off)) break;
            int sidx = -1;
            for (int sI = 0; sI < S; ++sI)
                if (slots[sI].phase == FREE) { sidx = sI; break; }
            if (sidx < 0) { arena.release(off, need[i]); break; }
            ++qhead;
            Slot& s = slots[sidx];
            s = Slot{};
            s.inst = i;
            s.c = ctx[i];
            s.b = b[i];
            s.x = x[i];
            s.off = off;
            s.bytes = need[i];
            const size_t nv = (size_t)s.c->nvec;
            unsigned char* p = arena.base + off;
            s.V = reinterpret_cast<double2*>(p);
            s.zt = s.V + (size_t)(m + 1) * nv;
            s.ut = s.zt + nv;
            s.partial = reinterpret_cast<double2*>(p + align_up((size_t)(m + 3) * nv * sizeof(double2)));
            s.nblk = reduction_blocks(s.c->nvec);
            s.phase = INIT;
            s.H.assign((size_t)(m + 1) * m, 0.0);
            s.R.assign((size_t)(m + 1) * m, 0.0);
            s.g.assign(m + 1, 0.0);
            s.sn.assign(m, 0.0);
            s.cs.assign(m, 0.0);
            s.hscale.assign(m + 2, 1.0);
            s.st.t_setup = s.c->t_setup_ms;
            s.t0 = std::chrono::steady_clock::now();
            active.push_back(sidx);   // x is zeroed by the INIT step's grouped copy
        }
        return SG_OK;
    };

    auto vt_base = [&](const Slot& s) {
        VecTask t{};
        t.n = s.c->nvec;
        t.nblocks = s.nblk;
        t.ldv = s.c->nvec;
        return t;
    };

    int rc = admit();
    if (rc) return rc;
    if (active.empty()) return fail(SG_ENOMEM, "batched solve: no instance fits the arena");

    while (!active.empty()) {
        for (auto* gp : {&g_copy, &g_lin, &g_xupd, &g_res, &g_mdot, &g_red1, &g_upd1, &g_red2, &g_updn, &g_redn,
                         &g_pcopy})
            gp->clear();
        g_apply.clear();
        for (auto& kv : g_spec) kv.second.clear();
        g_tri.clear();
        g_tri32.clear();
        for (auto& gg : g_fwd) gg.clear();
        for (auto& gg : g_inv) gg.clear();
        stg.reset();

        // slots in use are the lowest indices (admission takes the first free one): the
        // per-slot tables below and the coefficient copy-back cover slots [0, nslot) only
        int nslot = 0;
        for (int sI : active) nslot = std::max(nslot, sI + 1);
        // scales and least-squares coefficients of this step (device copies in the staging)
        for (int sI : active) {
            const Slot& s = slots[sI];
            std::copy(s.hscale.begin(), s.hscale.end(), hscale_tab.begin() + (size_t)sI * (m + 2));
            if (s.phase == END)
                for (int i = 0; i < s.k; ++i) y_tab[(size_t)sI * (m + 1) + i] = make_double2(s.y[i].real(), s.y[i].imag());
        }
        const size_t off_scale = stg.put(hscale_tab.data(), (size_t)nslot * (m + 2) * sizeof(double));
        const size_t off_y = stg.put(y_tab.data(), (size_t)nslot * (m + 1) * sizeof(double2));
        // device addresses are only known after ensure(); keep offsets and patch below
        auto dscale = [&](int sI) { return reinterpret_cast<const double*>(stg.dev + off_scale) + (size_t)sI * (m + 2); };
        auto dy = [&](int sI) { return reinterpret_cast<const double2*>(stg.dev + off_y) + (size_t)sI * (m + 1); };
        // the staging buffer may be reallocated by ensure(): size it generously first
        {
            const size_t per = sizeof(VecTask) * 12 + sizeof(ApplyArgs) + sizeof(TriTask) + 2 * sizeof(GemmTask) + 32 * 4;
            rc = stg.ensure(align_up(stg.used) + (size_t)active.size() * per + 128 * ALIGN * 2);
            if (rc) return rc;
        }
        unsigned char* const dev_before = stg.dev;

        // build the task tables
        std::vector<std::pair<int, const double2*>> pc_in;   // (slot, precond input)
        for (int sI : active) {
            Slot& s = slots[sI];
            const long long n = s.c->nvec;
            double2* coef = d_coef + (size_t)sI * CW;
            if (s.phase == INIT) {
                VecTask t = vt_base(s);
                t.x = s.b;
                t.a = make_double2(1, 0);
                t.w = s.V;
                g_copy.add(t, s.nblk, 32.0 * n);
                VecTask z = vt_base(s);   // x = 0 (no x, no y)
                z.a = make_double2(1, 0);
                z.w = s.x;
                g_copy.add(z, s.nblk, 16.0 * n);
            } else if (s.phase == END) {
                VecTask t = vt_base(s);
                t.V = s.V;
                t.nv = s.k;
                t.scale = dscale(sI);
                t.coef = dy(sI);
                t.w = s.ut;
                g_lin.add(t, s.nblk, 16.0 * (s.k + 1) * n);
                g_lin.maxnv = std::max(g_lin.maxnv, s.k);
                pc_in.push_back({sI, s.ut});
            } else if (s.phase == ARN) {
                pc_in.push_back({sI, s.V + (size_t)s.j * n});
            }
            (void)coef;
        }
        // preconditioner z = P^{-1} in  →  zt
        for (auto& pi : pc_in) {
            Slot& s = slots[pi.first];
            Ctx* c = s.c;
            const long long n = c->nvec;
            if (pc == SG_PC_NONE || c->dim == 1) {
                VecTask t = vt_base(s);
                t.x = pi.second;
                t.a = make_double2(1, 0);
                t.w = s.zt;
                g_pcopy.add(t, s.nblk, 32.0 * n);
            }
            if (pc == SG_PC_NONE) continue;
            const TriFactors& f = c->tri[pc == SG_PC_MEAN ? 0 : 1];
            if (c->dim == 1) {
                TriTask tt = make_tri_task(f, s.zt, c->n, c->n, c->Q, 1, tri_nr);
                g_tri.add(tt, tt.nblocks, 32.0 * n + 65.0 * f.nsys * c->n);
            } else {
                const int cfg = gemm_cfg_for(c->n, c->Q * c->n, prec);
                const int M = c->Q * c->n;
                GemmTask gf = make_gemm_task(prec, reinterpret_cast<const double*>(pi.second), c->n, c->fwd, c->n,
                                             reinterpret_cast<double*>(c->d_tmp_pc), c->tld, M, cfg);
                GemmTask gi = make_gemm_task(prec, reinterpret_cast<const double*>(c->d_tmp_pc), c->tld, c->inv, c->n,
                                             reinterpret_cast<double*>(s.zt), c->n, M, cfg);
                gf.io = t32 ? GEMM_IO_C32 : GEMM_IO_F64;
                gi.io = t32 ? GEMM_IO_A32 : GEMM_IO_F64;
                const double fl = (gemm_cfg_3m(cfg) ? 6.0 : 8.0) * M * (double)c->n * c->n;
                g_fwd[cfg].add(gf, gf.tiles_m * gf.tiles_n, fl);
                g_inv[cfg].add(gi, gi.tiles_m * gi.tiles_n, fl);
                TriTask tt = make_tri_task(f, c->d_tmp_pc, c->n, c->tld, c->Q, 2, t32 ? tri_nr32 : tri_nr);
                (t32 ? g_tri32 : g_tri).add(tt, tt.nblocks, (t32 ? 16.0 : 32.0) * n + 65.0 * f.nsys * c->n);
            }
        }
        size_t lds = 0;
        auto add_apply = [&](Ctx* c, const double2* xin, double2* yout) {
            const ApplyArgs aa = make_apply_args(c, xin, yout);
            const double abytes = (double)c->P * (32.0 * c->Q + 8.0 * c->K.nfield);
            if (c->dim == 2 && c->use_spec_apply && c->op_csl_beta == 0.0 &&
                (long long)c->n * c->n * 16 < (1ll << 32) &&
                dispatch_spec_grouped(c->s, c->degree, nullptr, nullptr, 0, 0, nullptr)) {
                g_spec[{c->s, c->degree}].add(aa, spec_row_blocks(c->n), abytes);
            } else {
                g_apply.add(aa, aa.ntiles_x * aa.nrows, abytes);
                lds = std::max(lds, apply_lds_bytes(c->Q, c->K.nfield));
            }
        };
        for (int sI : active) {
            Slot& s = slots[sI];
            Ctx* c = s.c;
            const long long n = c->nvec;
            double2* coef = d_coef + (size_t)sI * CW;
            if (s.phase == END) {
                VecTask t = vt_base(s);
                t.x = s.x;
                t.y = s.zt;
                t.a = make_double2(1, 0);
                t.b = make_double2(1, 0);
                t.w = s.x;
                g_xupd.add(t, s.nblk, 48.0 * n);
                add_apply(c, s.x, s.ut);
                VecTask r = vt_base(s);
                r.x = s.b;
                r.y = s.ut;
                r.a = make_double2(1, 0);
                r.b = make_double2(-1, 0);
                r.w = s.V;
                g_res.add(r, s.nblk, 48.0 * n);
            } else if (s.phase == ARN) {
                add_apply(c, s.zt, s.V + (size_t)(s.j + 1) * n);
                const int nv = s.j + 1;
                VecTask t = vt_base(s);
                t.V = s.V;
                t.nv = nv;
                t.scale = dscale(sI);
                t.w = s.V + (size_t)(s.j + 1) * n;
                t.partial = s.partial;
                VecTask md = t;
                g_mdot.add(md, s.nblk, 16.0 * (nv + 1) * n);
                VecTask r1 = t;
                r1.out = coef;
                g_red1.add(r1, nv);
                VecTask u1 = t;
                u1.coef = coef;
                g_upd1.add(u1, s.nblk, 16.0 * (nv + 2) * n);
                g_upd1.maxnv = std::max(g_upd1.maxnv, nv);
                VecTask r2 = t;
                r2.out = coef + nv;
                g_red2.add(r2, nv);
                VecTask un = t;
                un.coef = coef + nv;
                g_updn.add(un, s.nblk, 16.0 * (nv + 2) * n);
                g_updn.maxnv = std::max(g_updn.maxnv, nv);
                VecTask rn = t;
                rn.out = coef + 2 * nv;
                g_redn.add(rn, 1);
            }
            if (s.phase == INIT || s.phase == END) {
                VecTask un = vt_base(s);
                un.V = s.V;
                un.nv = 0;
                un.w = s.V;
                un.partial = s.partial;
                g_updn.add(un, s.nblk, 16.0 * n);
                VecTask rn = un;
                rn.out = coef;
                g_redn.add(rn, 1);
            }
        }

        // one upload of every table of the step
        for (auto* gp : {&g_copy, &g_lin, &g_pcopy, &g_xupd, &g_res, &g_mdot, &g_red1, &g_upd1, &g_red2, &g_updn,
                         &g_redn})
            stg.put_group(*gp);
        stg.put_group(g_apply);
        for (auto& kv : g_spec) stg.put_group(kv.second);
        stg.put_group(g_tri);
        stg.put_group(g_tri32);
        for (auto& gg : g_fwd) stg.put_group(gg);
        for (auto& gg : g_inv) stg.put_group(gg);
        if (stg.used > stg.cap || stg.dev != dev_before) return fail(SG_EINVAL, "batched solve: staging overflow");
        std::memcpy(stg.pinned, stg.host.data(), stg.used);
        SG_HIP(hipMemcpyAsync(stg.dev, stg.pinned, stg.used, hipMemcpyHostToDevice, stream));

        // launches, in dependency order
        if ((rc = launch_axpby_grouped(stg.dtasks(g_copy), stg.dstart(g_copy), g_copy.n(), g_copy.total(), g_copy.work,
                                       stream)))
            return rc;
        if ((rc = launch_lincomb_grouped(stg.dtasks(g_lin), stg.dstart(g_lin), g_lin.n(), g_lin.total(), g_lin.maxnv,
                                         g_lin.work, stream)))
            return rc;
        if ((rc = launch_axpby_grouped(stg.dtasks(g_pcopy), stg.dstart(g_pcopy), g_pcopy.n(), g_pcopy.total(),
                                       g_pcopy.work, stream)))
            return rc;
        for (int cfg = 0; cfg < SG_GEMM_NCFG; ++cfg)
            if ((rc = launch_gemm_grouped(prec, cfg, t32 ? GEMM_IO_C32 : GEMM_IO_F64, stg.dtasks(g_fwd[cfg]),
                                          stg.dstart(g_fwd[cfg]), g_fwd[cfg].n(), g_fwd[cfg].total(), g_fwd[cfg].work,
                                          stream)))
                return rc;
        int max_seg = 0, max_seg32 = 0;
        for (const TriTask& tt : g_tri.tasks) max_seg = std::max(max_seg, tt.f.L);
        for (const TriTask& tt : g_tri32.tasks) max_seg32 = std::max(max_seg32, tt.f.L);
        if ((rc = launch_tri_grouped(stg.dtasks(g_tri), stg.dstart(g_tri), g_tri.n(), g_tri.total(), max_seg, tri_nr,
                                     false, g_tri.work, stream)))
            return rc;
        if ((rc = launch_tri_grouped(stg.dtasks(g_tri32), stg.dstart(g_tri32), g_tri32.n(), g_tri32.total(), max_seg32,
                                     tri_nr32, true, g_tri32.work, stream)))
            return rc;
        for (int cfg = 0; cfg < SG_GEMM_NCFG; ++cfg)
            if ((rc = launch_gemm_grouped(prec, cfg, t32 ? GEMM_IO_A32 : GEMM_IO_F64, stg.dtasks(g_inv[cfg]),
                                          stg.dstart(g_inv[cfg]), g_inv[cfg].n(), g_inv[cfg].total(), g_inv[cfg].work,
                                          stream)))
                return rc;
        if ((rc = launch_axpby_grouped(stg.dtasks(g_xupd), stg.dstart(g_xupd), g_xupd.n(), g_xupd.total(), g_xupd.work,
                                       stream)))
            return rc;
        if ((rc = launch_apply_grouped(stg.dtasks(g_apply), stg.dstart(g_apply), g_apply.n(), g_apply.total(), lds,
                                       g_apply.work, stream)))
            return rc;
        for (auto& kv : g_spec) {
            Group<ApplyArgs>& gg = kv.second;
            if (gg.n() == 0) continue;
            KScope ks(SG_K_APPLY, gg.work, stream);
            dispatch_spec_grouped(kv.first.first, kv.first.second, stg.dtasks(gg), stg.dstart(gg), gg.n(), gg.total(),
                                  stream);
            SG_HIP(hipGetLastError());
        }
        if ((rc = launch_axpby_grouped(stg.dtasks(g_res), stg.dstart(g_res), g_res.n(), g_res.total(), g_res.work,
                                       stream)))
            return rc;
        if ((rc = launch_multidot_grouped(stg.dtasks(g_mdot), stg.dstart(g_mdot), g_mdot.n(), g_mdot.total(),
                                          g_upd1.maxnv, g_mdot.work, stream)))
            return rc;
        if ((rc = launch_reduce_grouped(stg.dtasks(g_red1), stg.dstart(g_red1), g_red1.n(), g_red1.total(), 0, stream)))
            return rc;
        if ((rc = launch_upd_grouped(stg.dtasks(g_upd1), stg.dstart(g_upd1), g_upd1.n(), g_upd1.total(), g_upd1.maxnv,
                                     true, g_upd1.work, stream)))
            return rc;
        if ((rc = launch_reduce_grouped(stg.dtasks(g_red2), stg.dstart(g_red2), g_red2.n(), g_red2.total(), 0, stream)))
            return rc;
        if ((rc = launch_upd_grouped(stg.dtasks(g_updn), stg.dstart(g_updn), g_updn.n(), g_updn.total(), g_updn.maxnv,
                                     false, g_updn.work, stream)))
            return rc;
        if ((rc = launch_reduce_grouped(stg.dtasks(g_redn), stg.dstart(g_redn), g_redn.n(), g_redn.total(), 1, stream)))
            return rc;
        SG_HIP(hipMemcpyAsync(h_coef, d_coef, (size_t)nslot * CW * sizeof(double2), hipMemcpyDeviceToHost, stream));
        if ((rc = wait_stream(stream, step_done))) return rc;

        // host part of every active instance
        std::vector<int> still;
        for (int sI : active) {
            Slot& s = slots[sI];
            const double2* hc = h_coef + (size_t)sI * CW;
            bool finished = false;
            if (s.phase == INIT) {
                const double beta = hc[0].x;
                if (!std::isfinite(beta)) {
                    s.st.relres_true = NAN;
                    finished = true;
                } else if (beta == 0.0) {
                    s.st.converged = 1;
                    s.st.relres_true = 0;
                    finished = true;
                } else {
                    s.bnorm = beta;
                    s.st.relres_true = 1.0;
                    s.hscale[0] = 1.0 / beta;
                    std::fill(s.g.begin(), s.g.end(), cd(0));
                    s.g[0] = beta;
                    s.j = 0;
                    s.phase = ARN;
                }
            } else if (s.phase == END) {
                const double beta = hc[0].x;
                ++s.st.restarts;
                s.st.relres_true = beta / s.bnorm;
                if (!std::isfinite(beta)) {
                    finished = true;
                } else if (s.st.relres_true <= o->tol) {
                    s.st.converged = 1;
                    finished = true;
                } else if (s.breakdown || s.st.iters >= o->maxit) {
                    finished = true;
                } else {
                    s.hscale[0] = 1.0 / beta;
                    std::fill(s.g.begin(), s.g.end(), cd(0));
                    s.g[0] = beta;
                    s.j = 0;
                    s.phase = ARN;
                }
            } else if (s.phase == ARN) {
                const int j = s.j;
                const double sj = s.hscale[j];
                double colnorm = 0;
                bool bad = false;
                for (int i = 0; i <= j; ++i) {
                    const double2 a1 = hc[i], a2 = hc[j + 1 + i];
                    const cd hv = sj * cd(a1.x + a2.x, a1.y + a2.y);
                    if (!std::isfinite(hv.real()) || !std::isfinite(hv.imag())) bad = true;
                    s.H[(size_t)i * m + j] = hv;
                    colnorm += std::norm(hv);
                }
                const double nrm = hc[2 * (j + 1)].x;
                if (bad || !std::isfinite(nrm)) {
                    s.st.relres_true = NAN;
                    finished = true;
                } else {
                    const double hnext = sj * nrm;
                    s.H[(size_t)(j + 1) * m + j] = hnext;
                    colnorm = std::sqrt(colnorm + hnext * hnext);
                    std::vector<cd> col(j + 2);
                    for (int i = 0; i <= j + 1; ++i) col[i] = s.H[(size_t)i * m + j];
                    for (int i = 0; i < j; ++i) {
                        const cd t = s.cs[i] * col[i] + s.sn[i] * col[i + 1];
                        col[i + 1] = -std::conj(s.sn[i]) * col[i] + s.cs[i] * col[i + 1];
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
                    s.cs[j] = cj;
                    s.sn[j] = sjr;
                    col[j] = cj * a + sjr * bb;
                    col[j + 1] = 0.0;
                    for (int i = 0; i <= j + 1; ++i) s.R[(size_t)i * m + j] = col[i];
                    s.g[j + 1] = -std::conj(sjr) * s.g[j];
                    s.g[j] = cj * s.g[j];
                    ++s.st.iters;
                    s.st.relres_est = std::abs(s.g[j + 1]) / s.bnorm;
                    s.breakdown = !(nrm > 1e-14 * colnorm / (sj > 0 ? sj : 1.0)) || hnext <= 1e-14 * colnorm;
                    const bool end = s.breakdown || s.st.relres_est <= o->tol || j + 1 == m || s.st.iters >= o->maxit;
                    if (!s.breakdown) s.hscale[j + 1] = 1.0 / nrm;
                    if (end) {
                        const int k = j + 1;
                        s.y.assign(k, 0.0);
                        for (int i = k - 1; i >= 0; --i) {
                            cd acc = s.g[i];
                            for (int l = i + 1; l < k; ++l) acc -= s.R[(size_t)i * m + l] * s.y[l];
                            s.y[i] = acc / s.R[(size_t)i * m + i];
                            if (!std::isfinite(s.y[i].real()) || !std::isfinite(s.y[i].imag())) bad = true;
                        }
                        if (bad) {
                            s.st.relres_true = NAN;
                            finished = true;
                        } else {
                            s.k = k;
                            s.phase = END;
                        }
                    } else {
                        s.j = j + 1;
                    }
                }
            }
            if (finished) {
                s.st.t_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - s.t0).count();
                if (!s.st.converged) any_notconv = true;
                if (stats) stats[s.inst] = s.st;
                arena.release(s.off, s.bytes);
                s.phase = FREE;
                ++ndone;
            } else {
                still.push_back(sI);
            }
        }
        active.swap(still);
        if ((rc = admit())) return rc;
        if (active.empty() && qhead < queue.size()) return fail(SG_ENOMEM, "batched solve: arena fragmentation");
    }
    (void)ndone;
    return any_notconv ? SG_ENOTCONV : SG_OK;
}

int batched_release() {
    int dev = 0;
    SG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) return fail(SG_EINVAL, "device index out of range");
    ArenaCache& ac = g_arena[dev];
    std::lock_guard<std::mutex> lk(ac.mu);
    if (ac.p) {
        SG_HIP(hipDeviceSynchronize());
        (void)hipFree(ac.p);
    }
    ac.p = nullptr;
    ac.bytes = 0;
    return SG_OK;
}

// Allocation of the per-handle buffers: when the device is full while an idle cached arena
// holds memory, the arena is returned first and the allocation tried once more. An arena
// that a batched solve is using (its lock held) is left alone.
hipError_t device_alloc(void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) return e;
    (void)hipGetLastError();
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return e;
    ArenaCache& ac = g_arena[dev];
    {
        std::unique_lock<std::mutex> lk(ac.mu, std::try_to_lock);
        if (!lk.owns_lock() || !ac.p) return e;
        (void)hipDeviceSynchronize();
        (void)hipFree(ac.p);
        ac.p = nullptr;
        ac.bytes = 0;
    }
    e = hipMalloc(p, bytes);
    if (e != hipSuccess) (void)hipGetLastError();
    return e;
}

// Autotuner: for every distinct (n, Q) of the 2D handles, time each GEMM tile shape on a
// grouped launch over up to `group` instances of that shape (the batched setting), and
// keep the fastest per instance in the process-wide table.
int autotune(int count, Ctx* const* ctx, int precision, int reps, double* ms_out, hipStream_t stream) {
    if (count < 0 || (count > 0 && !ctx)) return fail(SG_EINVAL, "bad handle list");
    if (precision < SG_PREC_F64 || precision > SG_PREC_BF16X3) return fail(SG_EINVAL, "unknown precision");
    if (reps < 1) reps = 3;
    std::map<std::pair<int, int>, std::vector<Ctx*>> classes;
    for (int i = 0; i < count; ++i) {
        if (!ctx[i]) return fail(SG_EINVAL, "null handle");
        if (ctx[i]->dim == 2 && !ctx[i]->vmean) classes[{ctx[i]->n, ctx[i]->Q}].push_back(ctx[i]);
    }
    hipEvent_t e0, e1;
    SG_HIP(hipEventCreate(&e0));
    SG_HIP(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } ev{e0, e1};
    double total_ms = 0;
    const int group = 8;
    for (auto& kv : classes) {
        const int n = kv.first.first, Q = kv.first.second;
        std::vector<Ctx*>& hs = kv.second;
        const int G = std::min<int>(group, (int)hs.size());
        const size_t nv = (size_t)hs[0]->nvec;
        double2* buf = nullptr;
        if (hipMalloc(&buf, (size_t)G * nv * sizeof(double2)) != hipSuccess)
            return fail(SG_ENOMEM, "autotune: scratch allocation failed");
        struct FB {
            double2* p;
            ~FB() { (void)hipFree(p); }
        } fb{buf};
        SG_HIP(hipMemsetAsync(buf, 0, (size_t)G * nv * sizeof(double2), stream));
        // tasks: the forward transform (zeroed scratch of task g -> the handle's own
        // intermediate) and the inverse one (intermediate -> scratch), the two layouts of a
        // preconditioner application, in two launches per repetition
        int* d_start = nullptr;
        GemmTask* d_tasks = nullptr;
        SG_HIP(hipMalloc(&d_start, 2 * (G + 1) * sizeof(int)));
        struct FS {
            void* p;
            ~FS() { (void)hipFree(p); }
        } fs{d_start};
        SG_HIP(hipMalloc(&d_tasks, 2 * G * sizeof(GemmTask)));
        struct FT {
            void* p;
            ~FT() { (void)hipFree(p); }
        } ft{d_tasks};
        double best = 1e300;
        int best_cfg = 0;
        for (int cfg = 0; cfg < SG_GEMM_NCFG; ++cfg) {
            if (!gemm_cfg_valid(cfg, precision)) continue;
            std::vector<GemmTask> tasks(2 * G);
            std::vector<int> start(2 * (G + 1), 0);
            for (int g = 0; g < G; ++g) {
                double* io = reinterpret_cast<double*>(buf + (size_t)g * nv);
                double* tmp = reinterpret_cast<double*>(hs[g]->d_tmp_pc);
                tasks[g] = make_gemm_task(precision, io, n, hs[g]->fwd, n, tmp, hs[g]->tld, Q * n, cfg);
                tasks[G + g] = make_gemm_task(precision, tmp, hs[g]->tld, hs[g]->inv, n, io, n, Q * n, cfg);
                if (precision != SG_PREC_F64) {   // the FP32 intermediate of the reduced-precision forms
                    tasks[g].io = GEMM_IO_C32;
                    tasks[G + g].io = GEMM_IO_A32;
                }
                start[g + 1] = start[g] + tasks[g].tiles_m * tasks[g].tiles_n;
                start[G + 1 + g + 1] = start[G + 1 + g] + tasks[G + g].tiles_m * tasks[G + g].tiles_n;
            }
            SG_HIP(hipMemcpyAsync(d_tasks, tasks.data(), 2 * G * sizeof(GemmTask), hipMemcpyHostToDevice, stream));
            SG_HIP(hipMemcpyAsync(d_start, start.data(), 2 * (G + 1) * sizeof(int), hipMemcpyHostToDevice, stream));
            auto both = [&]() {
                const bool r32 = precision != SG_PREC_F64;
                int rc = launch_gemm_grouped(precision, cfg, r32 ? GEMM_IO_C32 : GEMM_IO_F64, d_tasks, d_start, G,
                                             start[G], 0.0, stream);
                if (rc) return rc;
                return launch_gemm_grouped(precision, cfg, r32 ? GEMM_IO_A32 : GEMM_IO_F64, d_tasks + G,
                                           d_start + G + 1, G, start[2 * G + 1], 0.0, stream);
            };
            int rc = both();
            if (rc) return rc;
            SG_HIP(hipEventRecord(e0, stream));
            for (int r = 0; r < reps; ++r)
                if ((rc = both())) return rc;
            SG_HIP(hipEventRecord(e1, stream));
            SG_HIP(hipEventSynchronize(e1));
            float ms = 0;
            SG_HIP(hipEventElapsedTime(&ms, e0, e1));
            total_ms += ms;
            const double per = ms / (reps * (double)G);
            if (per < best) {
                best = per;
                best_cfg = cfg;
            }
        }
        tune_set(n, Q, precision, best_cfg);
    }
    if (ms_out) *ms_out = total_ms;
    return SG_OK;
}

}  // namespace sgi
