// Packed-row annealing kernels specialised to d = 27.  The
// specialised kernels are split over several translation units so that the
// large unrolled ones compile in parallel.
#include "xzzx_device.h"

namespace xzzx {

AnnealKernel static_rows_kernel_f(int d, bool plain)
{
    switch (d) {
    case 27: return plain ? k_anneal_rows_d_plain<27> : k_anneal_rows_d<27>;
    default: return nullptr;
    }
}

}  // namespace xzzx
