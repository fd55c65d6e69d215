"""RSM repetitive tasks on MI355X (gfx950): Python binding of librsm.

The data-parallel computation the paper's models describe -- a MARTE RSM
repetitive task (Sec. 3, Sec. 6.1, Sec. 7): tilers (origin, paving, fitting,
modular over the array shape) gather patterns, an elementary task runs once
per repetition, and a tiler scatters the results.  All of it runs in
hand-written HIP kernels behind the C-ABI declared in include/rsm.h; this
package only marshals torch tensors (device memory and streams) into that
ABI.
"""
from .rsm import (Batch, Chain, RsmError, TiledChain, TiledTask, indices, plan, run, run_adjoint,
                  run_chain, run_chain_adjoint, run_chain_train, run_csr, cg_solve, time_next_kernel, validate)

__all__ = ["Batch", "Chain", "RsmError", "TiledChain", "TiledTask", "indices", "plan", "run",
           "run_adjoint", "run_chain", "run_chain_adjoint", "run_chain_train", "run_csr", "cg_solve", "time_next_kernel", "validate"]
