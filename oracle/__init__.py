"""Plain, slow, FP64 CPU oracle for the parabolic-operator hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import or call this package; only the tests, the
small smoke check and the CPU-baseline leg of the benchmark use it.  It
shares no code with the GPU path: both consume the same seeded inputs from
the separate ``workloads`` package and nothing else.

Every function follows the paper (Caplan, Mikic, Linker & Lionello 2016,
"Advancing parabolic operators in thermodynamic MHD models") and cites the
passage it implements.  Where the paper is silent or garbled, the reading
taken is stated in the docstring.

Modules
  geometry  - finite-volume geometry of the logically rectangular grid
  operator  - the linearised conduction / viscosity operator F(u) = V^-1 (S u + g)
  rkl2      - RKL2 super-time-stepping (Fig. "rkl2", coefficient block, Eq. rkl2_s)
  pcg       - backward Euler + preconditioned CG (Eqs. BE..BE_linsolve, Fig. "pcg")
  ilu0      - non-overlapping block ILU0 preconditioner (Appendix A, PC2)
  rkl_variants - sub-cycled RKL2, Euler sub-steps, odd s and RKL1 (Sec. 6)
  nonlinear - conduction with kappa taken from the current state (no lagging)
  resistivity - edge-staggered curl curl A (Eq. mhd:a) and its BE + PC1 solve
  cnn       - FP64 reference of the small 3D CNN used for learned initial guesses
  learned_pc - the learned factored preconditioner M^-1 = G G^T: its entries,
              applications, training objective and gradient

Parity status: every function is pinned by the CPU tests in
tests/test_oracle_*.py (closed forms, invariants, brute force on tiny grids);
among them the block-ILU0 apply by dense solves of (L U) z = r per block
(ragged and 8^3 blocks) and Adam by its unrolled moment sums over several
steps with beta1 != beta2.
The conduction discretisation itself is a reading of the paper's "standard
scheme" (an exactly symmetric energy form with the same 19-point stencil);
its agreement with the paper's own scheme is parity unpinned, as no code or
data of that scheme exists here.
"""
