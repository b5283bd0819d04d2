"""Seeded synthetic inputs shared, as data only, by the oracle and the HIP path.

This package builds tight-binding Hamiltonians shaped like the paper's workloads
(a local-basis sparse symmetric H, Results section) and nothing else: it holds none
of the method's arithmetic (no graph, partition, expansion or density matrix).
"""
from .model import (  # noqa: F401
    CONFIGS,
    ModelSpec,
    make_model,
    make_operator_v,
    operator_v_pairs,
    displace_sites,
    rebuild_hamiltonian,
    ell_sha256,
)
