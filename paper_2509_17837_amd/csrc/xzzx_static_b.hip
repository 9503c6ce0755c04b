// Packed-row annealing kernels specialised to d = 15, 17.  The
// specialised kernels are split over several translation units so that the
// large unrolled ones compile in parallel.
#include "xzzx_device.h"

namespace xzzx {

AnnealKernel static_rows_kernel_b(int d, bool plain)
{
    switch (d) {
    case 15: return plain ? k_anneal_rows_d_plain<15> : k_anneal_rows_d<15>;
    case 17: return plain ? k_anneal_rows_d_plain<17> : k_anneal_rows_d<17>;
    default: return nullptr;
    }
}

}  // namespace xzzx
