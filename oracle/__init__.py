"""Plain FP64 CPU oracle of the nDGP multigrid hot path (arXiv:1511.08200).

TEST INFRASTRUCTURE ONLY: used by the tests, the package's smoke check and
the benchmark's CPU-baseline leg, never by the solver.  It shares no code
with the HIP path."""
