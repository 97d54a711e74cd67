"""MI355X (gfx950) greedy binary code construction (arXiv:1507.05398).

The computation lives in ``libgreedy_code.so`` (hand-written HIP, C ABI in
``include/greedy_code.h``); this package only marshals arguments to it.
"""
from ._native import (EXPORTS, GC_BORDER, GC_EBUSY, GC_ECAPACITY, GC_EDEVICE, GC_EINVAL, GC_ENOMEM,
                      GC_ETIMEOUT, GC_GRAY, GC_GREVLEX, GC_GRLEX, GC_JOB_ADMITTED, GC_JOB_DONE,
                      GC_JOB_FAILED, GC_JOB_WAITING, GC_LEX, GC_OK, ORDERINGS, GreedyCodeError,
                      BatchGraph, BatchPlan, Server, device_code, gc_last_error, gc_version, greedy_code,
                      greedy_code_batch, greedy_code_capacity, greedy_code_device,
                      greedy_code_device_ex, greedy_code_device_noalloc, greedy_code_cw64, greedy_code_tune, greedy_code_tune_reset, load,
                      GcProblem, problem, problem_positions, problem_capacity, greedy_code_problem,
                      greedy_code_problem_device, device_problem_code, probe_block_loop, probe_matrix_loop,
                      probe_barrier)

__all__ = ["EXPORTS", "GC_BORDER", "GC_EBUSY", "GC_ECAPACITY", "GC_EDEVICE", "GC_EINVAL", "GC_ENOMEM",
           "GC_ETIMEOUT", "GC_GRAY", "GC_GREVLEX", "GC_GRLEX", "GC_JOB_ADMITTED", "GC_JOB_DONE",
           "GC_JOB_FAILED", "GC_JOB_WAITING", "GC_LEX", "GC_OK", "ORDERINGS", "GreedyCodeError",
           "BatchGraph", "BatchPlan", "Server", "device_code", "gc_last_error", "gc_version", "greedy_code",
           "greedy_code_batch", "greedy_code_capacity", "greedy_code_device",
           "greedy_code_device_ex", "greedy_code_device_noalloc", "greedy_code_cw64", "greedy_code_tune", "greedy_code_tune_reset", "load",
           "GcProblem", "problem", "problem_positions", "problem_capacity", "greedy_code_problem",
           "greedy_code_problem_device", "device_problem_code", "probe_block_loop", "probe_matrix_loop",
           "probe_barrier"]
