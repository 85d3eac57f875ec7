// Instantiations of the shape-specialised SG operator: (3, 4), (3, 3), (4, 2), (2, 4).
#include "apply_spec.inc"

namespace sgi {
int dispatch_spec_g2(int s, int r, const ApplyArgs& a, hipStream_t st) {
    SG_SPEC(3, 4)
    SG_SPEC(3, 3)
    SG_SPEC(4, 2)
    SG_SPEC(2, 4)
    return 0;
}
int dispatch_spec_grouped_g2(int s, int r, const ApplyArgs* d, const int* ds, int nt, int tot, hipStream_t st) {
    SG_SPEC_G(3, 4)
    SG_SPEC_G(3, 3)
    SG_SPEC_G(4, 2)
    SG_SPEC_G(2, 4)
    return 0;
}
}  // namespace sgi
