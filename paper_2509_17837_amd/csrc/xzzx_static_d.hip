// Packed-row annealing kernels specialised to d = 23.  The
// specialised kernels are split over several translation units so that the
// large unrolled ones compile in parallel.
#include "xzzx_device.h"

namespace xzzx {

AnnealKernel static_rows_kernel_d(int d, bool plain)
{
    switch (d) {
    case 23: return plain ? k_anneal_rows_d_plain<23> : k_anneal_rows_d<23>;
    default: return nullptr;
    }
}

}  // namespace xzzx
