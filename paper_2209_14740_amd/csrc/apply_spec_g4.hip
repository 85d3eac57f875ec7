// Instantiations of the shape-specialised SG operator: (3, 5), (3, 6), (3, 7), (3, 8), the
// high-degree shapes of three random variables (2D; Q = 56, 84, 120, 165).
#include "apply_spec.inc"

namespace sgi {
int dispatch_spec_g4(int s, int r, const ApplyArgs& a, hipStream_t st) {
    SG_SPEC(3, 5)
    SG_SPEC(3, 6)
    SG_SPEC(3, 7)
    SG_SPEC(3, 8)
    return 0;
}
int dispatch_spec_grouped_g4(int s, int r, const ApplyArgs* d, const int* ds, int nt, int tot, hipStream_t st) {
    SG_SPEC_G(3, 5)
    SG_SPEC_G(3, 6)
    SG_SPEC_G(3, 7)
    SG_SPEC_G(3, 8)
    return 0;
}
}  // namespace sgi
