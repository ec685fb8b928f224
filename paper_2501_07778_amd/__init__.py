"""MI355X QTT finite element hot path: Python binding of libqtt.so.

The binding only marshals arguments: every step of the computation runs in
the library's HIP kernels.  PyTorch provides device memory (the caller-owned
core buffers and workspaces of the C ABI) and the stream.  Importing the
package loads the library and fails loudly when it is missing.
"""
from ._lib import (  # noqa: F401
    LIB_PATH, QttError, TT, Problem, SolveOpts, lib, load_library,
    matvec, matvec_round, matvec_round_workspace, round_, round_sketch, dot, dot_noalloc, kernel_timing, kernel_timing_read, tt_combine, tt_align, tt_contract_last, axpby, assemble, assemble_bpx, solve, solve_workspace_bytes,
    tt_from_cores, tt_to_cores, problem_from_workload, version,
    Batch, solve_batched, autotune_batched, StepBatch, StepGraph, matvec_round_batched,
    MLP, columns, tt_from_packed,
)
