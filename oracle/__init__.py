"""CPU FP64 oracle of the damped Gauss-Newton hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg import or run anything in this package; the GPU
library and its Python binding never do, and they share no code with it.
Only the seeded input generators (package `workloads`) feed both sides.

Contents:
- profile1d: geometry, tanh-MLP jets, envelope, Hilbert term, CCF / local
  Burgers residual rows, parameter Jacobian by a reverse sweep (numpy).
- dense (dense.c): compensated Gram and gradient, textbook Cholesky, forward
  and back substitution (plain C, built with gcc).
- gn: the damped Gauss-Newton step composed from the two.

Every function is pinned by tests/test_oracle_*.py against closed forms,
complex-step derivatives, brute force or library routines, never against the
GPU path.
"""
