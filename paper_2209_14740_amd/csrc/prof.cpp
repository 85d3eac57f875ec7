// Per-kernel-class timing with HIP events on the launch stream (sg_set_profiling).
#include <hip/hip_runtime.h>

#include "sg_internal.h"

namespace sgi {

thread_local Prof* g_prof = nullptr;

hipEvent_t Prof::get() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    // timing only: no system-scope release at the event, which would write back and
    // invalidate caches between the kernels it separates
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

void Prof::begin(hipStream_t st, hipEvent_t* ev) {
    *ev = get();
    if (*ev && hipEventRecord(*ev, st) != hipSuccess) *ev = nullptr;
}

void Prof::end(int kind, double w, hipStream_t st, hipEvent_t ev) {
    hipEvent_t b = get();
    if (!b || hipEventRecord(b, st) != hipSuccess) return;
    pending.push_back(Rec{ev, b, kind, w});
    if (pending.size() > 16384) resolve();
}

int Prof::resolve() {
    for (auto& r : pending) {
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(SG_EHIP, "event synchronisation failed");
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
            ms[r.kind] += t;
            cnt[r.kind] += 1;
            work[r.kind] += r.work;
        }
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    pending.clear();
    return SG_OK;
}

void Prof::reset() {
    resolve();
    for (int k = 0; k < SG_K_NKINDS; ++k) {
        ms[k] = 0;
        cnt[k] = 0;
        work[k] = 0;
    }
}

Prof::~Prof() {
    for (auto& r : pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
}

}  // namespace sgi
