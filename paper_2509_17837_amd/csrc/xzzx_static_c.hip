// Packed-row annealing kernels specialised to d = 19, 21.  The
// specialised kernels are split over several translation units so that the
// large unrolled ones compile in parallel.
#include "xzzx_device.h"

namespace xzzx {

AnnealKernel static_rows_kernel_c(int d, bool plain)
{
    switch (d) {
    case 19: return plain ? k_anneal_rows_d_plain<19> : k_anneal_rows_d<19>;
    case 21: return plain ? k_anneal_rows_d_plain<21> : k_anneal_rows_d<21>;
    default: return nullptr;
    }
}

}  // namespace xzzx
