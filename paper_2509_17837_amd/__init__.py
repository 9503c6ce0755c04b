"""MI355X (gfx950) simulated-annealing decoder for the XZZX surface code
(arXiv:2509.17837).  The computation lives in libxzzx_sa.so (C ABI in
include/xzzx_sa.h); `decoder` is its thin Python binding."""

__all__ = ["decoder", "inputs", "build"]
