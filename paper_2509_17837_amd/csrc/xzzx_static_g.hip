// Packed-row annealing kernels specialised to d = 29.  The
// specialised kernels are split over several translation units so that the
// large unrolled ones compile in parallel.
#include "xzzx_device.h"

namespace xzzx {

AnnealKernel static_rows_kernel_g(int d, bool plain)
{
    switch (d) {
    case 29: return plain ? k_anneal_rows_d_plain<29> : k_anneal_rows_d<29>;
    default: return nullptr;
    }
}

}  // namespace xzzx
