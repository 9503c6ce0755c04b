// Replica-exchange kernels specialised to the rotated lattice at d = 17, 19,
// 21, 23 (two words per row; the core is in xzzx_ladder_rows.h).
#include "xzzx_ladder_rows.h"

namespace xzzx {

AnnealKernel ladder_rows_kernel_c(int d, bool plain);

AnnealKernel ladder_rows_kernel_large(int d, bool plain)
{
    switch (d) {
    case 17: return plain ? k_anneal_ladder_rows_d_plain<17> : k_anneal_ladder_rows_d<17>;
    case 19: return plain ? k_anneal_ladder_rows_d_plain<19> : k_anneal_ladder_rows_d<19>;
    case 21: return plain ? k_anneal_ladder_rows_d_plain<21> : k_anneal_ladder_rows_d<21>;
    case 23: return plain ? k_anneal_ladder_rows_d_plain<23> : k_anneal_ladder_rows_d<23>;
    default: return ladder_rows_kernel_c(d, plain);
    }
}

}  // namespace xzzx
