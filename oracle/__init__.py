"""FP64 CPU checker for the FC^2T^2 hot path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark may import
anything from this package.  The product path (the HIP library and its Python binding)
never does; it shares no code, table or helper with this package.  Inputs come from the
seeded generators in ``paper_2111_00110_amd.workloads``, which hold no arithmetic of the
method.

Two parts:

* ``direct``  -- the exact O(NM) sums the method approximates (paper eq. (1) in section 3,
  the explicit layer of section 4, the line integral of section 6.1, the ray root of
  section 5), with their gradients, in FP64.
* ``fmm``/``rays`` -- the method itself, step by step in the paper's order and notation
  (P2M, M2M, M2L with the parity window and the near-field hole, L2L, L2P; their exact
  transposes for the backward pass; line-to-polynomial, ray integration, ray insertion and
  root finding on the local expansions), in FP64 numpy.

``kernels`` gives the kernel functions and their partial derivatives: Hermite closed forms
for the Gaussian, sympy differentiation for the inverse multiquadric, exact monomial
differentiation for polynomial test kernels.
"""
