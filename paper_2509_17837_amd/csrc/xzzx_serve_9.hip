// Serving kernel of the specialised packed-row family for d = 9
// (one register class; the kernel branches on the task's distance).  Each
// class lives in its own translation unit so that they compile in parallel.
#include "xzzx_device.h"

namespace xzzx {

ServeKernel serve_class_kernel_9() { return k_serve_rows_class<9, 9>; }

}  // namespace xzzx
