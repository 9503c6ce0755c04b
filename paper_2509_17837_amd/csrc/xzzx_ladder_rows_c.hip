// Replica-exchange kernels specialised to the rotated lattice at d = 25, 27,
// 29, 31 (two words per row; the core is in xzzx_ladder_rows.h).
#include "xzzx_ladder_rows.h"

namespace xzzx {

AnnealKernel ladder_rows_kernel_c(int d, bool plain)
{
    switch (d) {
    case 25: return plain ? k_anneal_ladder_rows_d_plain<25> : k_anneal_ladder_rows_d<25>;
    case 27: return plain ? k_anneal_ladder_rows_d_plain<27> : k_anneal_ladder_rows_d<27>;
    case 29: return plain ? k_anneal_ladder_rows_d_plain<29> : k_anneal_ladder_rows_d<29>;
    case 31: return plain ? k_anneal_ladder_rows_d_plain<31> : k_anneal_ladder_rows_d<31>;
    default: return nullptr;
    }
}
static_assert(kLadderRowsMaxD == 31, "the ladder kernels instantiate d = 3 .. 31");

}  // namespace xzzx
