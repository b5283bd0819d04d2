"""CPU oracle for graph-based linear-scaling density matrices (test infrastructure).

This package is a plain, slow, obviously correct CPU implementation of what the
GPU library computes, written from the paper (Niklasson et al., "Graph-based linear
scaling electronic structure theory") in FP64 with numpy / scipy / LAPACK.  It is
test infrastructure only: the test suite, the smoke check and the benchmark's CPU
baseline may use it; the library itself never imports, links or calls it, and it
shares no code with the library (only the seeded input generator in ``synth``).

Modules
  bounds       Gershgorin spectral bounds and the SP2 start map X0
  graph        data-dependency graphs (Eq. 2 with the X0^2 estimate; Eq. 8)
  partition    cores (communities) and core+halo subgraphs (Eq. 6, obs. vi)
  sp2          gather, partitioned SP2 (the parity reference), whole-matrix
               thresholded SP2, column assembly of D
  exact        dense diagonalisation: D = occupied eigenprojector
  equivalence  Eq. 3-6: whole-matrix masked polynomial vs subgraph polynomials
  adjoint      reverse-mode derivative of Tr[D V] through the SP2 recursion
  foe          finite-temperature Chebyshev Fermi-operator expansion per subgraph (Eq. 7)
  metrics      error measures of Fig. 2 (Frobenius per site, band energy)

Parity pins: every function is checked in tests/ against closed forms, brute force,
invariants or the paper's equivalence; see the module docstrings.
"""
