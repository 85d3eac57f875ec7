// Instantiations of the shape-specialised SG operator: (4, 4), (4, 3).
#include "apply_spec.inc"

namespace sgi {
int dispatch_spec_g1(int s, int r, const ApplyArgs& a, hipStream_t st) {
    SG_SPEC(4, 4)
    SG_SPEC(4, 3)
    return 0;
}
int dispatch_spec_grouped_g1(int s, int r, const ApplyArgs* d, const int* ds, int nt, int tot, hipStream_t st) {
    SG_SPEC_G(4, 4)
    SG_SPEC_G(4, 3)
    return 0;
}
}  // namespace sgi
