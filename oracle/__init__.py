"""CPU reference ("oracle") for the sketch-preconditioned infeasible IPM.

TEST INFRASTRUCTURE ONLY.  Plain, slow, FP64 NumPy/SciPy code written from the
paper (Chowdhury, London, Avron, Drineas, "Speeding up Linear Programming using
Randomized Linear Algebra").  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the GPU library never does, and it
shares no code with it.  The only thing both sides share is the seeded input
generator package `lpgen`, which holds none of the method's arithmetic.

Modules
  sketch  the sparse embedding W (counter-based hash written out from its
          definition)
  ipm     Alg. 2 (infeasible long-step IPM) with an exact Cholesky solve of the
          normal equations ("IPM w/ Dir." of the experiments), and with Alg. 1
          (sketch-preconditioned CG through Q^{-1/2} from an SVD) plus the
          correction vector v; the step-length rule; residuals and invariants
  vertex  brute-force vertex enumeration for tiny LPs
"""
