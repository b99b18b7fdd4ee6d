"""CPU FP64 oracle of the damped Gauss-Newton hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg import or run anything in this package; the GPU
library and its Python binding never do, and they share no code with it.
Only the seeded input generators (package `workloads`) feed both sides.

Contents:
- profile1d: geometry, tanh-MLP jets, envelope, Hilbert term, CCF / local
  Burgers residual rows, parameter Jacobian by a reverse sweep (numpy).
- profile2d: 2D coordinates, second-order network jets in y (Taylor mode),
  IPM-style and Boussinesq-type residual rows, parameter Jacobian by the
  complex-step derivative (numpy).
- deriv1d: d1 and d2 loss rows of the 1D problems (Taylor-mode field
  derivatives to third order, odd and even half-line Hilbert quadrature,
  complex-step Jacobian).
- stage2: second stage of multi-stage training (equation linearised around a
  fixed first stage, Fourier feature network, complex-step Jacobian).
- dense (dense.c): compensated Gram and gradient, textbook Cholesky, forward
  and back substitution (plain C, built with gcc).
- gn: the damped Gauss-Newton step composed from the two, and the step with
  Levenberg-Marquardt damping.
- rank1: the stochastic full-matrix Gauss-Newton step (moving average of
  rank-1 curvature estimates, closed-form learning rate and momentum).
- funnel: funnel inference of lam (the signed residual proxy near the origin
  and the secant update).

Every function is pinned by tests/test_oracle_*.py against closed forms,
complex-step derivatives, brute force or library routines, never against the
GPU path.
"""
