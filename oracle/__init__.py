"""FP64 CPU oracle for the JGS2 per-iteration solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import or call anything in this package; only tests, the
smoke check and the CPU-baseline leg of the benchmark do.  It shares no code
with the HIP path; only the seeded input generators
(``paper_2506_06494_amd.inputs``) serve both.

Every function is a plain, slow, direct transcription of what the paper
(Lan et al., "JGS2: Near Second-order Converging Jacobi/Gauss-Seidel for GPU
Elastodynamics", arXiv 2506.06494) defines, in float64, with numpy/scipy
primitives (dense and banded LAPACK factorisations, SVD, symmetric
eigensolvers, NNLS) as single steps.  Where the paper is silent or
ambiguous, the reading taken is stated at the function.

Modules:
  snh        stable Neo-Hookean energy density, stress and stress differential
  fem        tet kinematics, lumped mass, incremental potential, gradient,
             element Hessians, sparse assembly, plane barriers
  newton     global projected-Newton reference solve (sparse direct)
  mesh       adjacency and greedy vertex colouring
  rng        counter-based SplitMix64 draws used by cubature training
  correction rest Hessian, co-rotated basis U-bar, training poses, cubature
  sweep      per-vertex local systems (variants R0, R1, R2, R2G1, R3, P0), Jacobi and
             coloured Gauss-Seidel sweeps, the time-step loop
  adjoint    implicit-function adjoint of the time-step map

Parity status: every function is pinned by a CPU test against closed forms,
finite differences, brute force or library routines, except where its
docstring says "parity unpinned".
"""
