"""MI355X (gfx950) implementation of the fast Grover-search simulation of arXiv:2005.04635.

The work happens in libgrover.so (HIP kernels behind the C ABI of include/grover.h); this package holds its
sources (csrc/), its build script (build.py) and the ctypes binding (grover.py). Nothing is loaded at import
time; the first call that needs the library loads it and fails loudly when it has not been built.
"""
from .grover import (  # noqa: F401
    EXPORTS,
    Grover,
    GroverBatch,
    GroverError,
    grover_apply_hadamard_all,
    grover_batch_capture,
    grover_batch_config,
    grover_batch_destroy,
    grover_batch_init,
    grover_batch_last_error,
    grover_batch_query,
    grover_batch_read_state,
    grover_batch_run,
    grover_batch_set_tiling,
    grover_batch_state,
    grover_batch_sync,
    grover_batch_tune,
    grover_config,
    grover_destroy,
    grover_gate_iterate,
    grover_init,
    grover_iterate,
    grover_last_error,
    grover_marked,
    grover_norm,
    grover_optimal_iterations,
    grover_query,
    grover_read_state,
    grover_reset,
    grover_sample,
    grover_sample_u53,
    grover_state_device,
    grover_status_str,
    grover_sync,
    grover_write_state,
    load,
)
