// Shared declarations of the SG operator kernels (generic and shape-specialised).
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "sg_internal.h"

namespace sgi {

struct ApplyArgs {
    const double2* x;
    double2* y;
    const double* D2;
    const double* D1;
    const int* prog;
    const double* vals;
    long long P;
    int n, Q, ng2, ng1, dim;
    double ih2;
    int kpp, kpj, ktp, ktf, bpp, bpj, btp, btf, kv, bv;
    int ntiles_x, nrows;
    const double* KF;     // k_1..k_s at the nodes ([s][P]) for the shape-specialised kernels
    double k0, ih;        // constant mean k_0 and 1/h
    const double* K0;     // k_0 at the nodes when it varies in space (null: the constant k0)
    double csl_beta;      // 0: the operator A; β: the shifted operator M(β) = A - iβK (k² block times 1+iβ)
};

ApplyArgs make_apply_args(const Ctx* c, const double2* x, double2* y);
size_t apply_lds_bytes(int Q, int ng2);
// Generic operator over many (x, y, operator) tasks; task t owns tiles [start[t], start[t+1])
// (n_tiles = ntiles_x · nrows); lds is the largest apply_lds_bytes of the tasks.
int launch_apply_grouped(const ApplyArgs* d_tasks, const int* d_start, int ntask, int total, size_t lds,
                         double bytes, hipStream_t st);

// Shape-specialised operator launchers, one translation unit per group of (s, r)
// shapes (apply_spec_g*.hip); each returns 1 if it handled (s, r), else 0.
int dispatch_spec_g0(int s, int r, const ApplyArgs& a, hipStream_t st);
int dispatch_spec_g1(int s, int r, const ApplyArgs& a, hipStream_t st);
int dispatch_spec_g2(int s, int r, const ApplyArgs& a, hipStream_t st);
int dispatch_spec_g3(int s, int r, const ApplyArgs& a, hipStream_t st);
int dispatch_spec_g4(int s, int r, const ApplyArgs& a, hipStream_t st);
// Grouped forms over tasks of one shape (2D); with d == nullptr only report availability.
// Task t needs spec_row_blocks(n) blocks.
int dispatch_spec_grouped_g0(int s, int r, const ApplyArgs* d, const int* ds, int nt, int tot, hipStream_t st);
int dispatch_spec_grouped_g1(int s, int r, const ApplyArgs* d, const int* ds, int nt, int tot, hipStream_t st);
int dispatch_spec_grouped_g2(int s, int r, const ApplyArgs* d, const int* ds, int nt, int tot, hipStream_t st);
int dispatch_spec_grouped_g3(int s, int r, const ApplyArgs* d, const int* ds, int nt, int tot, hipStream_t st);
int dispatch_spec_grouped_g4(int s, int r, const ApplyArgs* d, const int* ds, int nt, int tot, hipStream_t st);
inline int dispatch_spec_grouped(int s, int r, const ApplyArgs* d, const int* ds, int nt, int tot, hipStream_t st) {
    return dispatch_spec_grouped_g0(s, r, d, ds, nt, tot, st) || dispatch_spec_grouped_g1(s, r, d, ds, nt, tot, st) ||
           dispatch_spec_grouped_g2(s, r, d, ds, nt, tot, st) || dispatch_spec_grouped_g3(s, r, d, ds, nt, tot, st) ||
           dispatch_spec_grouped_g4(s, r, d, ds, nt, tot, st);
}
inline int spec_row_blocks(int n) { return ((n + 31) / 32) * ((n + 3) / 4); }

}  // namespace sgi
