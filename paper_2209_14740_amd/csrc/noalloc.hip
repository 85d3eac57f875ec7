// sg_cgs2_noalloc: one CGS2 step (the kernels of sg_cgs2) for callers that cannot
// allocate device memory.  The reduction partials and the coefficients live in a
// file-scope device array instead of buffers allocated per call.
//
// In host code the array's name is only a host-side stand-in, not a device address:
// its address on a device is looked up once per device (hipGetSymbolAddress, with that
// device current) and only that address is passed to kernels and copies.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "sg_internal.h"

namespace sgi {
namespace {

constexpr int NA_MAXNV = 64;                                        // basis vectors per call
constexpr int NA_MAXBLK = 2048;                                     // first-stage reduction blocks
constexpr long long NA_PARTIAL = (long long)NA_MAXBLK * NA_MAXNV;   // partial sums [block][k]
constexpr long long NA_ELEMS = NA_PARTIAL + 3 * NA_MAXNV;           // + 2nv+1 coefficients

// 2 MiB + 3 KiB per device, held until the process ends.
__device__ __align__(256) double2 scratch[NA_ELEMS];

// Device address of this device's scratch array (looked up on the first call per device).
int scratch_ptr(double2** out) {
    constexpr int MAXDEV = 64;
    static std::mutex mu;
    static double2* ptr[MAXDEV] = {};
    int dev = -1;
    SG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAXDEV) return fail(SG_EINVAL, "sg_cgs2_noalloc: device index out of range");
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        SG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SG_EHIP, "sg_cgs2_noalloc: no device address for the scratch array");
        ptr[dev] = static_cast<double2*>(p);
    }
    *out = ptr[dev];
    return SG_OK;
}

}  // namespace

static int cgs2_noalloc(long long n, int nv, const double2* V, double2* w, double2* h_host, hipStream_t st) {
    if (nv > NA_MAXNV)
        return fail(SG_EINVAL, "sg_cgs2_noalloc: nv = " + std::to_string(nv) + " is above the limit of " +
                                   std::to_string(NA_MAXNV) + " basis vectors of its fixed scratch array");
    const int nb = reduction_blocks(n);
    if (nb > NA_MAXBLK) return fail(SG_EINVAL, "sg_cgs2_noalloc: reduction grid above the scratch array");
    double2* base = nullptr;
    int rc = scratch_ptr(&base);
    if (rc) return rc;
    double2* partial = base;             // nb·nv partial sums (every entry written before it is read)
    double2* coef = base + NA_PARTIAL;   // 2nv+1 coefficients
    double2 hbuf[2 * NA_MAXNV + 1];      // pageable host copy of the coefficients
    rc = cgs2_step(n, nv, V, n, nullptr, w, partial, nb, coef, hbuf, st);   // synchronises st
    if (rc) return rc;
    const double nrm = hbuf[2 * nv].x;
    for (int k = 0; k < nv; ++k) h_host[k] = make_double2(hbuf[k].x + hbuf[nv + k].x, hbuf[k].y + hbuf[nv + k].y);
    h_host[nv] = make_double2(nrm, 0.0);
    if (!std::isfinite(nrm)) return fail(SG_ENONFINITE, "non-finite norm");
    if (nrm > 0.0) {
        if ((rc = launch_scale_copy(n, 1.0 / nrm, w, w, st))) return rc;
        SG_HIP(hipStreamSynchronize(st));
    }
    return SG_OK;
}

}  // namespace sgi

extern "C" int sg_cgs2_noalloc(long long n, int nv, const sg_c64* V, sg_c64* w, sg_c64* h_host, hipStream_t stream) {
    try {
        if (n < 1 || nv < 1 || !V || !w || !h_host) return sgi::fail(SG_EINVAL, "invalid argument");
        return sgi::cgs2_noalloc(n, nv, reinterpret_cast<const double2*>(V), reinterpret_cast<double2*>(w),
                                 reinterpret_cast<double2*>(h_host), stream);
    } catch (...) {
        return sgi::fail(SG_EINVAL, "unexpected exception");
    }
}
