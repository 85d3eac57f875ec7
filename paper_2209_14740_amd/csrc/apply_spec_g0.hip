// Instantiations of the shape-specialised SG operator: (6, 3).
#include "apply_spec.inc"

namespace sgi {
int dispatch_spec_g0(int s, int r, const ApplyArgs& a, hipStream_t st) {
    SG_SPEC(6, 3)
    return 0;
}
int dispatch_spec_grouped_g0(int s, int r, const ApplyArgs* d, const int* ds, int nt, int tot, hipStream_t st) {
    SG_SPEC_G(6, 3)
    return 0;
}
}  // namespace sgi
