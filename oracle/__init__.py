"""CPU FP64 oracle for the batched multiphase chemistry solve.

THIS PACKAGE IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it. The product path (the HIP library and its
Python binding) never imports, calls or links anything here, and nothing here imports
the product path.

It is a plain, slow, obviously correct implementation of what the method computes:

* ``expand``  -- phase x instance expansion of a mechanism into a flat list of
  generalized mass-action reactions over one state vector (Sect. 2.2.3, AerosolPhase).
* ``rates``   -- rate constants from the environment (Table of Process classes).
* ``forcing`` -- f(y) and the analytic dense Jacobian (Sect. 2.4.2, the two sums over
  process contributions).
* ``bdf``     -- variable-order, variable-step BDF with Newton iteration and a dense
  partial-pivot LU (Sect. 2.4.1 names CVODE's BDF + Newton; the formulas follow the
  published backward-difference form of Shampine & Reichelt 1997, with kappa = 0).
* ``sparse``  -- brute-force boolean symbolic elimination and a no-pivot dense LU in a
  given order, used to pin the host compiler's fill and the device LU.
* ``solve``   -- per-cell driver tying these together.

Parity of the full configurations against the paper is unpinned (the paper prints no
result values); every function here is pinned by the CPU tests in tests/test_oracle_*.py.
"""
