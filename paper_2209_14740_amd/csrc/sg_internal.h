// Internal declarations shared by the host setup, the solver drivers and the kernel
// launch wrappers of the SG Helmholtz library.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "sg.h"

namespace sgi {

using cplx = std::complex<double>;

void set_error(const std::string& msg);
const char* last_error();
int fail(int code, const std::string& msg);

#define SG_HIP(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess)                                                     \
            return ::sgi::fail(SG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Host→device uploads of a setup.  They go through a non-blocking stream that SetupStream
// creates for the calling thread's setup (the null stream outside one) and each is complete
// when the call returns, so a setup neither queues behind nor waits for solves that other
// threads run meanwhile (synchronous copies on the null stream can do both).
struct SetupStream {
    SetupStream();
    ~SetupStream();
    int rc;   // SG_OK, or the error of creating the stream
};
int upload(void* dst, const void* src, size_t bytes);
int upload_zero(void* dst, size_t bytes);
// Time a setup spends in device allocations, uploads and its stream (milliseconds, the calling
// thread's current setup; reported by sg_setup_times).
struct SetupClock {
    double alloc = 0, upload = 0, stream = 0;
};
SetupClock& setup_clock();
hipError_t setup_alloc_raw(void** p, size_t bytes);
template <class T>
hipError_t setup_alloc(T** p, size_t bytes) {
    return setup_alloc_raw(reinterpret_cast<void**>(p), bytes);
}

// Coupling program of the matrix-free operator.  For output block i the pairs
// [pair_ptr[i], pair_ptr[i+1]) list the input blocks j with a nonzero coupling; pair p
// owns terms [term_ptr[p], term_ptr[p+1]) = (field index γ, triple-product value G_γ[i,j]).
struct Coupling {
    int nfield = 0;                     // number of coefficient fields
    std::vector<int> pair_ptr;          // Q+1
    std::vector<int> pair_j;            // npairs
    std::vector<int> term_ptr;          // npairs+1
    std::vector<int> term_field;        // nterms
    std::vector<double> term_val;       // nterms
};

// One pivoted tridiagonal LU factorisation per system (row-partial pivoting).
// Arrays are indexed [row * nsys + sys] so that consecutive systems are contiguous.
struct TriFactors {
    int len = 0, nsys = 0;
    double2* dl = nullptr;    // multipliers l_i (row i+1 minus l_i * row i), len-1 rows
    double2* dinv = nullptr;  // 1 / u_ii
    double2* du1 = nullptr;   // u_{i,i+1}
    double2* du2 = nullptr;   // u_{i,i+2}
    uint8_t* piv = nullptr;   // 1 if rows i and i+1 were swapped at step i
    // segmented form (rows split into K <= 32 segments of L <= 16 rows up to n = 512, see precond.hip)
    int K = 0, L = 0;
    double2* u1p = nullptr;   // u_{i,i+1} / u_ii   (len rows, zero past the end)
    double2* u2p = nullptr;   // u_{i,i+2} / u_ii
    double2* phi = nullptr;   // forward propagator of segment k: [k][sys]
    double2* psi = nullptr;   // backward 2x2 propagator of segment k: [k][sys][4]
    uint32_t* pivm = nullptr; // row-exchange flags of segment k as bits u = i - k·L: [k][sys]
};

// Expanded real form of a complex N×N matrix for the GEMM C = A·B, where A rows are
// complex-interleaved: Bexp[2k+c][2n+d] with c,d ∈ {0,1} (see precond.hip).
struct DenseB {
    double* f64 = nullptr;     // [2N][2N]
    float* f32 = nullptr;      // [2N][2N]
    uint16_t* bf_hi = nullptr; // [2N][2N] bf16 bits, packed for the MFMA B operand
    uint16_t* bf_lo = nullptr;
    double* p3 = nullptr;      // 3M planes of B (n-major [n][k], ld = bexp_ld(N)): Re, Im
    float* p3f = nullptr;      // the same in FP32
};

// One dense problem C[M][Nc] = A[M][Kc] · B of the preconditioner transforms, Bt[Nc][Kc]
// n-major in the compute precision; A and C are FP64 (complex interleaved).
struct GemmTask {
    const double* A;
    const void* Bt0;
    const void* Bt1;
    double* C;
    long long lda, ldb, ldc;
    int M, Nc, Kc, tiles_m, tiles_n;
    // element types of A and C in the FP32 and BF16x3 forms (FP64 ignores it): GEMM_IO_F64
    // both FP64; GEMM_IO_C32 C stored as FP32 (the forward transform into the FP32
    // intermediate); GEMM_IO_A32 A read as FP32 (the inverse transform out of it).  A and C
    // keep their FP64 pointer types; lda and ldc count elements of the stored type.
    int io = 0;
};
enum { GEMM_IO_F64 = 0, GEMM_IO_C32 = 1, GEMM_IO_A32 = 2 };
// GEMM tile shapes: the expanded real form (BM × BN real columns, every precision) 0:
// 128×128, 1: 64×128, 2: 64×64, 3: 64×32, 4: 32×64, 9: 64×256, 10: 128×256 (FP32 / BF16x3);
// the 3M complex form (BM × BN complex columns, FP64 and FP32) 5: 32×32, 6: 64×32, 7: 32×64,
// 8: 64×64.
enum { SG_GEMM_NCFG = 11 };
inline bool gemm_cfg_3m(int cfg) { return cfg >= 5 && cfg <= 8; }
inline bool gemm_cfg_valid(int cfg, int precision) {
    if (cfg < 0 || cfg >= SG_GEMM_NCFG) return false;
    if (gemm_cfg_3m(cfg)) return precision == SG_PREC_F64 || precision == SG_PREC_F32;
    if (cfg >= 9) return precision != SG_PREC_F64;
    return true;
}

// One set of tridiagonal solves: element i of system (q, a) is X[q*sq + a*sa + i*se],
// the factors of system a are at column a*fa of f.
struct TriTask {
    double2* X;
    TriFactors f;
    int len, na, nq, fa;
    long long se, sa, sq;
    int nblocks;
};

// One vector operation of a grouped launch (one solve of a batch).  Fields not used by
// an operation are ignored.
struct VecTask {
    const double2* V;        // basis vectors V_k = V + k*ldv
    long long ldv;
    const double* scale;     // v_k = scale[k] V_k (device, may be null = 1)
    const double2* coef;     // update / combination coefficients (device)
    double2* w;              // vector updated in place (update, norm) or written (axpby)
    const double2* x;        // axpby operands: w = a x + b y (y may be null)
    const double2* y;
    double2 a, b;
    double2* partial;        // first-stage partial sums [block][nout]
    double2* out;            // second-stage results
    long long n;             // vector length
    int nv;                  // number of basis vectors
    int nblocks;             // blocks of the first-stage kernels
};

// One instance's delayed-CGS2 step in a grouped launch (batched solver).  The basis holds the
// orthonormal v_0..v_{j-1} in slots 0..j-1, the candidate u_j in slot j and, for a full step,
// w_j = A z_j in slot j+1; the update pass overwrites slot j with v_j and slot j+1 with
// u_{j+1}.
struct DcgsTask {
    const double2* V;
    long long ldv, n;
    double2* partial;   // first-stage sums [block][2j+3] (finishing step: [block][j+1])
    double2* red;       // their totals
    double2* h1;        // first-pass projection of the previous step (j+1 entries)
    double2* rec;       // the step's record for the host (2j+3 entries)
    double2* cv;        // update coefficients (j, j and 2 entries)
    double2* cw;
    double2* cu;
    int j;              // basis vectors before the candidate
    int full;           // 1: w_j present; 0: finishing reduction of u_j alone (no update)
    int nblocks;        // first-stage blocks of this task
};

struct Workspace {
    int m = 0;                 // restart length the buffers were sized for
    bool flexible = false;
    double2* V = nullptr;      // (m+1) vectors
    double2* Z = nullptr;      // m vectors (flexible only)
    double2* tmp = nullptr;    // 2 scratch vectors
    double* scale = nullptr;   // m+1 lazy normalisation factors (device)
    double2* coef = nullptr;   // device coefficient buffer (2*(m+2) complex)
    double2* partial = nullptr;// reduction partials
    int npartial_blocks = 0;
    double2* host_pinned = nullptr; // pinned host mirror of coef
    hipEvent_t done = nullptr; // host waits of the Arnoldi loop poll this event
    // delayed CGS2 driver (dcgs2.cpp): reduction partials, small device arrays, pinned records
    int dm = 0;
    double2* dpart = nullptr;
    double2* dsmall = nullptr;
    double2* hrec = nullptr;
    double2* hrec_dev = nullptr;   // hrec's device address: the coefficient kernel writes the records there
};

// Optional per-kernel-class event timing (sg_set_profiling / sg_kernel_times).
struct Prof {
    bool on = false;
    unsigned mask = ~0u;            // kinds recorded when on (bit k = kind k)
    double ms[SG_K_NKINDS] = {};
    long long cnt[SG_K_NKINDS] = {};
    double work[SG_K_NKINDS] = {};
    struct Rec { hipEvent_t a, b; int kind; double work; };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    hipEvent_t get();
    void begin(hipStream_t st, hipEvent_t* ev);
    void end(int kind, double work, hipStream_t st, hipEvent_t ev);
    int resolve();
    void reset();
    ~Prof();
};
extern thread_local Prof* g_prof;

// RAII scope around one kernel launch: records events when profiling is on.
struct KScope {
    int kind;
    double work;
    hipStream_t st;
    hipEvent_t ev = nullptr;
    KScope(int k, double w, hipStream_t s) : kind(k), work(w), st(s) {
        if (g_prof && g_prof->on && ((g_prof->mask >> k) & 1u)) g_prof->begin(st, &ev);
    }
    ~KScope() {
        if (ev && g_prof && g_prof->on) g_prof->end(kind, work, st, ev);
    }
};

struct Net;

struct Ctx {
    int dim = 0, n = 0, s = 0, degree = 0, Q = 0;
    long long P = 0, nvec = 0;
    double h = 0, kbar = 0, beta = 0;
    int device = 0;
    std::vector<int> alpha;            // Q*s multi-indices

    Coupling K;                        // k² coupling (fields D2_γ = w·κ2_γ)
    Coupling B;                        // boundary k coupling (fields D1_γ = (e/h)·κ1_γ)
    std::vector<std::vector<int>> gamma2, gamma1;   // multi-indices of the fields

    // device copies
    double* d_D2 = nullptr;            // [K.nfield][P]
    double* d_D1 = nullptr;            // [B.nfield][P]
    int* d_prog = nullptr;             // packed integer tables (K then B)
    double* d_vals = nullptr;          // packed term values (K then B)
    int kprog_pairptr = 0, kprog_pairj = 0, kprog_termptr = 0, kprog_termfield = 0;
    int bprog_pairptr = 0, bprog_pairj = 0, bprog_termptr = 0, bprog_termfield = 0;
    int kvals_off = 0, bvals_off = 0;
    int out_order_off = 0;             // output block order (load balance)
    double* d_w = nullptr;             // node weights w (n^dim)
    std::vector<double> w_host;        // the same on the host (right-hand sides)
    double* d_kf = nullptr;            // k_1..k_s at the nodes ([s][P])

    // mean-block fast diagonalisation (x direction) and y-direction tridiagonal factors
    std::vector<cplx> Vt;              // eigenvectors, column a = v_a (N×N, row-major [x][a])
    std::vector<cplx> mu;              // eigenvalues of (T - iτE)v = μ D v
    DenseB fwd, inv;                   // B operands for R·Ṽ and W·Ṽᵀ
    TriFactors tri[2];                 // [0]: mean value A_0, [1]: mean CSL M_0

    Workspace ws;
    Prof prof;
    bool use_spec_apply = true;        // compile-time-specialised operator when available
    double op_csl_beta = 0.0;          // operator of sg_apply and the solvers: A (0) or M(β) = A - iβK
    double2* d_tmp_pc = nullptr;       // preconditioner intermediate: Q·n rows of tld complex (2D)
    int tld = 0;                       // its row length, n rounded up to 8 (128-byte aligned rows)
    // block solves by the exact block LU over the grid lines: a spatially varying mean k_0
    // (k_mean = 0 at setup), or the fallback when the eigenfactors fail their checks
    bool vmean = false;
    bool eig_fallback = false;         // line factorisation chosen because of the eigenfactors
    double cond_v = 0;                 // estimated cond₂ of the eigenvector matrix (2D, constant k̄)
    double* d_k0 = nullptr;            // k_0 at the nodes for the operator (null: constant kbar)
    int line_L = 0, line_nl = 0;       // line length and number of lines
    double2* d_lineE[2] = {};          // inverses of the line Schur complements, [j][k][i], A_0 and M_0
    double* d_lineb = nullptr;         // diagonal of the line coupling B
    double line_check[2] = {};         // setup residual of the factorisation (A_0, M_0)
    Net* net = nullptr;                // attached correction network (not owned)
    bool classic_cgs2 = false;         // sg_set_orthogonalisation(SG_ORTH_CGS2): the two-pass driver
    int last_k = 0;                    // orthonormal basis vectors of the last delayed-CGS2 cycle
    double t_setup_ms = 0;
    double t_setup_alloc_ms = 0, t_setup_upload_ms = 0, t_setup_stream_ms = 0;   // parts of t_setup_ms

    ~Ctx();
};

// setup.cpp
int build_ctx(const sg_problem* prob, hipStream_t stream, Ctx** out);
double eigen_cond_limit();
void set_eigen_cond_limit(double v);

// apply.hip
int launch_apply(const Ctx* c, const double2* x, double2* y, hipStream_t st);
// true if some operator kernel serves the handle's shape with the operator shift csl_beta
bool apply_available(const Ctx* c, double csl_beta);

// batched.cpp (autotuner table)
int tune_get(int n, int Q, int precision);
void tune_set(int n, int Q, int precision, int cfg);

// stats.hip (statistics of the solution)
int launch_moments(const Ctx* c, const double2* x, double2* mean, double* var, hipStream_t st);
int degree_magnitudes(const Ctx* c, const double2* x, double* gamma, hipStream_t st);

// line.hip (block solves with a spatially varying mean)
int build_line_factors(Ctx* c, const double* k0_host);
int launch_line(Ctx* c, int pc, const double2* r, double2* z, hipStream_t st);

// precond.hip
int launch_precond(Ctx* c, int pc, int precision, const double2* r, double2* z, hipStream_t st);
int upload_dense_b(Ctx* c, hipStream_t st);
void gemm_tiles(int cfg, int M, int Nc, int* tiles_m, int* tiles_n);
// tile shape of a transform with N×N operator and M rows: the autotuner's choice, else a
// size-based default
int gemm_default_cfg(int N, int M, int precision);
int gemm_cfg_for(int N, int M, int precision);
// lda, ldc: row lengths of A and C in complex elements
GemmTask make_gemm_task(int precision, const double* A, long long lda, const DenseB& B, int N, double* C,
                        long long ldc, int M, int cfg);
// io: GEMM_IO_*, the same for every task of the launch
int launch_gemm_grouped(int precision, int cfg, int io, const GemmTask* d_tasks, const int* d_start, int ntask,
                        int total, double flops, hipStream_t st);
// ld: row length of X in complex elements (2D; the 1D layout is contiguous); nr: right-hand
// sides per thread (2 only where tri_nr_ok holds), the same for every task of one launch
TriTask make_tri_task(const TriFactors& f, double2* X, int n, int ld, int Q, int dim, int nr = 1);
bool tri_nr_ok(const TriFactors& f, int n, int Q, int dim);
bool tri_nr_ok32(const TriFactors& f, int n, int Q, int dim);   // the same for an FP32 intermediate
// f32: every task's X is an FP32 (float2) intermediate
int launch_tri_grouped(const TriTask* d_tasks, const int* d_start, int ntask, int total, int max_seg, int nr,
                       bool f32, double bytes, hipStream_t st);

// krylov.hip
int ensure_workspace(Ctx* c, int m, bool flexible);
int launch_multidot(long long n, int nv, const double2* V, long long ldv, const double* scale,
                    const double2* w, double2* partial, int nblocks, hipStream_t st);
int launch_reduce(int nblocks, int nv, const double2* partial, const double* scale, double2* out,
                  hipStream_t st);
int launch_axpy_dot(long long n, int nv, const double2* V, long long ldv, const double* scale,
                    const double2* coef, double2* w, double2* partial, int nblocks, bool with_dot,
                    hipStream_t st);
int launch_norm2(long long n, const double2* x, double2* partial, int nblocks, hipStream_t st);
int launch_upd(long long n, int nv, const double2* V, long long ldv, const double* scale, const double2* coef,
               double2* w, double2* partial, int nblocks, bool dot, hipStream_t st);
// out[0] = (||.||, 0); inv (device, may be null) receives 1/||.||
int launch_reduce_norm(int nblocks, const double2* partial, double2* out, hipStream_t st, double* inv = nullptr);
int launch_lincomb(long long n, int nv, const double2* V, long long ldv, const double* scale,
                   const double2* coef, double2* x, hipStream_t st);
int launch_axpby(long long n, double2 a, const double2* x, double2 b, const double2* y, double2* out,
                 hipStream_t st);
int launch_scale_copy(long long n, double a, const double2* x, double2* out, hipStream_t st);
int reduction_blocks(long long n);
// Delayed CGS2 (see krylov.hip): reduction (w may be null: only a and α), coefficients, update.
int launch_dcgs_reduce(long long n, int nv, const double2* V, long long ldv, const double2* u, const double2* w,
                       double2* partial, int nblocks, double2* red, hipStream_t st);
int launch_dcgs_finalize(int j, bool full, const double2* red, double2* h1prev, double2* rec, double2* cv, double2* cw,
                         double2* cu, hipStream_t st);
int launch_dcgs_update(long long n, int nv, const double2* V, long long ldv, double2* u, double2* w, const double2* cv,
                       const double2* cw, const double2* cu, int nblocks, hipStream_t st);
// Grouped forms: task t of d_tasks owns blocks [start[t], start[t+1]) of the launch.
int launch_multidot_grouped(const VecTask* d_tasks, const int* d_start, int ntask, int total, int maxnv, double bytes,
                            hipStream_t st);
int launch_reduce_grouped(const VecTask* d_tasks, const int* d_start, int ntask, int total, int mode,
                          hipStream_t st);
int launch_upd_grouped(const VecTask* d_tasks, const int* d_start, int ntask, int total, int maxnv, bool dot,
                       double bytes, hipStream_t st);
int launch_dcgs_reduce_grouped(const DcgsTask* d_tasks, const int* d_start, int ntask, int total, int maxj, double bytes,
                               hipStream_t st);
int launch_dcgs_sum_grouped(const DcgsTask* d_tasks, const int* d_start, int ntask, int total, hipStream_t st);
int launch_dcgs_finalize_grouped(const DcgsTask* d_tasks, int ntask, hipStream_t st);
int launch_dcgs_update_grouped(const DcgsTask* d_tasks, const int* d_start, int ntask, int total, int maxj, double bytes,
                               hipStream_t st);
int launch_lincomb_grouped(const VecTask* d_tasks, const int* d_start, int ntask, int total, int maxnv,
                           double bytes, hipStream_t st);
int launch_axpby_grouped(const VecTask* d_tasks, const int* d_start, int ntask, int total, double bytes,
                         hipStream_t st);

// batched.cpp
int run_gmres_batched(int count, Ctx* const* ctx, const double2* const* b, double2* const* x,
                      const sg_solve_opts* o, sg_solve_stats* stats, hipStream_t stream);
int autotune(int count, Ctx* const* ctx, int precision, int reps, double* ms_out, hipStream_t stream);
int batched_release();
hipError_t device_alloc(void** p, size_t bytes);
int tune_get(int n, int Q, int precision);
void tune_set(int n, int Q, int precision, int cfg);

// net.cpp
int net_precond(Net* n, Ctx* c, int precision, const double2* v, double2* z, hipStream_t st);

// gmres.cpp
// wait for the work queued on st: poll ev (recorded here) when given, else block
int wait_stream(hipStream_t st, hipEvent_t ev);
int run_gmres(Ctx* c, const double2* b, double2* x, const sg_solve_opts* o, sg_precond_cb cb,
              void* user, bool flexible, sg_solve_stats* st, hipStream_t stream);
int run_stationary(Ctx* c, const double2* b, double2* x, int pc, int iters, double* hist, hipStream_t st);
// dcgs2.cpp: the delayed-CGS2 driver of the built-in right preconditioners (restart <= 64)
bool dcgs2_serves(const Ctx* c, const sg_solve_opts* o, sg_precond_cb cb);
int run_gmres_dcgs2(Ctx* c, const double2* b, double2* x, const sg_solve_opts* o, sg_solve_stats* st,
                    hipStream_t stream);
// d_next_scale (device, may be null) receives 1/||w|| after the two passes; the host waits
// for the coefficients by polling `done` (null: a blocking stream synchronisation); with
// wait = false (and done given) it only records `done` after the copy
int cgs2_step(long long n, int nv, const double2* V, long long ldv, const double* d_scale,
              double2* w, double2* partial, int nblocks, double2* d_coef, double2* h_pinned,
              hipStream_t st, double* d_next_scale = nullptr, hipEvent_t done = nullptr, bool wait = true);

}  // namespace sgi
