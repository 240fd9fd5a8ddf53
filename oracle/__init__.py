"""FP64 CPU oracle for the compressed history integrals.  TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference implementations of what the device
library computes, written from the paper's definitions:

  weights      exact-rational polynomial / Adams-Moulton / Gregory / Newton-Cotes
               weights (appendix "Integral and derivative approximations")
  history      dense O(N^3) history sums I^R and I^< (KBE right-hand sides,
               equations for the retarded and lesser components)
  closed_form  closed-form convolutions of damped exponentials (pins only)
  tsvd         truncated SVD with the absolute epsilon_SVD rule
               (section "Hierarchical decomposition")
  adjoint      dense gradient of the adjoint loss
  step_solve   the retarded time step (Volterra step solve) and its march
  born         the lattice second-Born self-energy of one time step

Only tests, the smoke entry point and the benchmark's CPU-baseline leg may
import this package.  The device library never calls it, links it or falls
back to it.  It shares no code with the device library; the only common
module is the seeded input generator `kbe_inputs`, which holds no method
arithmetic.
"""
