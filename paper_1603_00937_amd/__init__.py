"""Graph-partitioned SP2 density matrices on MI355X (Python binding of libgb).

Every step runs in the HIP library ``libgb.so``; this package only marshals torch
device tensors (memory) and the current HIP stream into the C ABI of include/gb.h.
"""
from .api import (  # noqa: F401
    GbError, Graph, Partition, Tape, DensityFn, spectral_bounds, build_graph, partition, density,
    density_with_grad, version, TorchAllocator, set_allocator, foe_density, chebyshev_fermi,
    foe_solve_mu, sp2_sequence, sp2_estimate_gap, gap_inputs, build_graph_rcut, trim,
    partition_host, partition_update, partition_update_host, density_workspace,
    spectral_bounds_noalloc, tune_save, tune_load, peak_rate,
)
