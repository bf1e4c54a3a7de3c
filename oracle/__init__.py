"""Plain FP64 CPU oracle for the immersed-boundary projection method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: it exists so that tests, the smoke check and the
benchmark's CPU baseline can compare the HIP library against a slow,
obviously correct implementation written directly from the paper
(Layton, Krishnan & Barba, "cuIBM -- A GPU-accelerated Immersed Boundary
Method", arXiv:1109.3524).  It shares no code with the HIP library; the only
common module is the synthetic input generator
(`paper_1109_3524_amd.workloads`), which holds none of the method's
arithmetic.

Modules
  grid       staggered-grid metrics (Sec. 2, staggered non-uniform grid)
  delta      Roma et al. discrete delta, interpolation matrix E (Sec. 2, Eqs. 5-7)
  operators  D, G, M, R, L, A, B^1, Q, K = Q^T B^1 Q (Sec. 2, Eqs. 8-11)
  flow       boundary values, convection, right-hand sides, one time step
  solvers    PCG, Jacobi preconditioner, smoothed-aggregation AMG (Sec. 3)
  dense      brute-force dense references for tiny grids

Every floating-point quantity is FP64.  Where the paper leaves a detail
open, the reading adopted is stated at the function that implements it.
"""
