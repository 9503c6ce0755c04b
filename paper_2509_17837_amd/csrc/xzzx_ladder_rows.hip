// Replica-exchange kernels specialised to the rotated lattice at d = 3, 5,
// ..., 15 (the core is in xzzx_ladder_rows.h), and the dispatch over every
// specialised distance.
#include "xzzx_ladder_rows.h"

namespace xzzx {

int ladder_rows_state_words(int d)
{
    return (d * (2 * (d + 1) <= 32 ? 1 : 2) + 3) / 4 * 4;
}

AnnealKernel ladder_rows_kernel(int d, bool plain)
{
    switch (d) {
    case 3: return plain ? k_anneal_ladder_rows_d_plain<3> : k_anneal_ladder_rows_d<3>;
    case 5: return plain ? k_anneal_ladder_rows_d_plain<5> : k_anneal_ladder_rows_d<5>;
    case 7: return plain ? k_anneal_ladder_rows_d_plain<7> : k_anneal_ladder_rows_d<7>;
    case 9: return plain ? k_anneal_ladder_rows_d_plain<9> : k_anneal_ladder_rows_d<9>;
    case 11: return plain ? k_anneal_ladder_rows_d_plain<11> : k_anneal_ladder_rows_d<11>;
    case 13: return plain ? k_anneal_ladder_rows_d_plain<13> : k_anneal_ladder_rows_d<13>;
    case 15: return plain ? k_anneal_ladder_rows_d_plain<15> : k_anneal_ladder_rows_d<15>;
    default: return ladder_rows_kernel_large(d, plain);
    }
}

}  // namespace xzzx
