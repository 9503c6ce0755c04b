// Serving kernel of the specialised packed-row family for d = 17, 19, 21
// (one register class; the kernel branches on the task's distance).  Each
// class lives in its own translation unit so that they compile in parallel.
#include "xzzx_device.h"

namespace xzzx {

ServeKernel serve_class_kernel_21() { return k_serve_rows_class<21, 17, 19, 21>; }

}  // namespace xzzx
