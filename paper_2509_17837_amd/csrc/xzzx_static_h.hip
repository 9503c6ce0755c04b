// Packed-row annealing kernels specialised to d = 31.  The
// specialised kernels are split over several translation units so that the
// large unrolled ones compile in parallel.
#include "xzzx_device.h"

namespace xzzx {

AnnealKernel static_rows_kernel_h(int d, bool plain)
{
    switch (d) {
    case 31: return plain ? k_anneal_rows_d_plain<31> : k_anneal_rows_d<31>;
    default: return nullptr;
    }
}

}  // namespace xzzx
