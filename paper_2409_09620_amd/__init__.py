"""MI355X-native BP RI-OEDG stage (Ding, Cui and Wu, arXiv 2409.09620).

The stage runs in hand-written HIP kernels behind the C ABI declared in
include/oedg.h; `binding` marshals arguments to it with ctypes and uses PyTorch
only for device memory and streams.
"""

from .binding import (DG_OE_CW, DG_OE_RI, Batch, DgError, Solver, host_mesh_tables, lib_path, load_library,
                      plan_chunks, symbols_declared)

__all__ = ["Solver", "Batch", "DgError", "host_mesh_tables", "plan_chunks", "DG_OE_RI", "DG_OE_CW", "load_library",
           "lib_path", "symbols_declared"]
