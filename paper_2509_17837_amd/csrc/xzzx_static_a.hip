// Packed-row annealing kernels specialised to d = 3, 5, 7, 9, 11, 13.  The
// specialised kernels are split over several translation units so that the
// large unrolled ones compile in parallel.
#include "xzzx_device.h"

namespace xzzx {

AnnealKernel static_rows_kernel_a(int d, bool plain)
{
    switch (d) {
    case 3: return plain ? k_anneal_rows_d_plain<3> : k_anneal_rows_d<3>;
    case 5: return plain ? k_anneal_rows_d_plain<5> : k_anneal_rows_d<5>;
    case 7: return plain ? k_anneal_rows_d_plain<7> : k_anneal_rows_d<7>;
    case 9: return plain ? k_anneal_rows_d_plain<9> : k_anneal_rows_d<9>;
    case 11: return plain ? k_anneal_rows_d_plain<11> : k_anneal_rows_d<11>;
    case 13: return plain ? k_anneal_rows_d_plain<13> : k_anneal_rows_d<13>;
    default: return nullptr;
    }
}

}  // namespace xzzx
