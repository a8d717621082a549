// Fine level of the two-level hierarchical far field (Sec. 5.2): dispatch
// to the kernel of the plan's order (pmmm_hier_cell.h, one compile unit per
// order).
#include "pmmm_hier.h"

namespace pmmm {

hipError_t launch_hier_m2l_f32(const HierArgs &a, hipStream_t s) {
    switch (a.p) {
        case 0: return hier_cell_launch<0>(a, s);
        case 1: return hier_cell_launch<1>(a, s);
        case 2: return hier_cell_launch<2>(a, s);
        case 3: return hier_cell_launch<3>(a, s);
        case 4: return hier_cell_launch<4>(a, s);
        case 5: return hier_cell_launch<5>(a, s);
        case 6: return hier_cell_launch<6>(a, s);
        case 7: return hier_cell_launch<7>(a, s);
        case 8: return hier_cell_launch<8>(a, s);
        case 9: return hier_cell_launch<9>(a, s);
        case 10: return hier_cell_launch<10>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pmmm
