// Instantiations of the shape-specialised SG operator: (1, 1), (1, 2), (1, 3), (1, 4), (1, 5), (2, 1), (2, 2), (2, 3), (3, 2).
#include "apply_spec.inc"

namespace sgi {
int dispatch_spec_g3(int s, int r, const ApplyArgs& a, hipStream_t st) {
    SG_SPEC(1, 1)
    SG_SPEC(1, 2)
    SG_SPEC(1, 3)
    SG_SPEC(1, 4)
    SG_SPEC(1, 5)
    SG_SPEC(2, 1)
    SG_SPEC(2, 2)
    SG_SPEC(2, 3)
    SG_SPEC(3, 2)
    return 0;
}
int dispatch_spec_grouped_g3(int s, int r, const ApplyArgs* d, const int* ds, int nt, int tot, hipStream_t st) {
    SG_SPEC_G(1, 1)
    SG_SPEC_G(1, 2)
    SG_SPEC_G(1, 3)
    SG_SPEC_G(1, 4)
    SG_SPEC_G(1, 5)
    SG_SPEC_G(2, 1)
    SG_SPEC_G(2, 2)
    SG_SPEC_G(2, 3)
    SG_SPEC_G(3, 2)
    return 0;
}
}  // namespace sgi
