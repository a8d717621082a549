// Internal declarations of the two-level hierarchical far field (Sec. 5.2):
// the fine level's table of singular harmonics and its local M2L.  Not part
// of the public ABI.
#pragma once

#include "pmmm_internal.h"

namespace pmmm {

// S_n^k (real storage, orders n <= 2p, cell units) at every fine offset d
// with |d_a| <= D, zero on the near cube max|d_a| <= cutoff; layout
// [((dz + D) W + dy + D) W + dx + D][Q], W = 2D + 1 (FP64 sums, FP32 values).
hipError_t build_hier_table_f32(int p, int cutoff, int D, float *out, hipStream_t s);

struct HierArgs {
    int p, nf, r, cutoff, D;   // fine mesh nf^3 = (coarse n r)^3, margin D = (c + 1) r - 1
    const float *M;            // fine moments [P(+1)][nf^3], cell units
    float *L;                  // fine local expansions [P][nf^3], written in full
    const float *table;        // build_hier_table_f32
};
hipError_t launch_hier_m2l_f32(const HierArgs &a, hipStream_t s);

// The fine-level kernel of one order (pmmm_hier_cell.h; instantiated for
// 0 <= PO <= PMMM_PMAX by pmmm_hier_inst.hip).
template <int PO>
hipError_t hier_cell_launch(const HierArgs &a, hipStream_t s);

}  // namespace pmmm
