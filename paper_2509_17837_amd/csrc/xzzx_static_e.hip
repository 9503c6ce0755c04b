// Packed-row annealing kernels specialised to d = 25.  The
// specialised kernels are split over several translation units so that the
// large unrolled ones compile in parallel.
#include "xzzx_device.h"

namespace xzzx {

AnnealKernel static_rows_kernel_e(int d, bool plain)
{
    switch (d) {
    case 25: return plain ? k_anneal_rows_d_plain<25> : k_anneal_rows_d<25>;
    default: return nullptr;
    }
}

}  // namespace xzzx
