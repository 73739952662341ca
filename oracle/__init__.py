"""CPU oracle for the cavity-DFTB hot path: TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 numpy code written from the paper (arXiv 2512.03277) and from
the standard second-order SCC-DFTB formulation it cites (Computational details:
DFTB with second-order self-consistent-charge correction).  It shares no code
with the HIP path and imports nothing from it.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import or run it; the product path
never does.

Modules
  sk       Slater-Koster H0 / S blocks and their analytic derivatives
  gamma    Elstner gamma function and its radial derivative
  scc      SCC loop (Broyden mixer), energy, forces, charges, dipole
  born     Mulliken and central-finite-difference Born charges
  cavity   multimode cavity: mode functions, dipole sums, fields, free rotation
  md       the velocity-Verlet-like cavity MD step of the paper (Step 1 + Step 3)
  harmonic harmonic matter backend used to pin the integrator
  surrogate descriptors / MLP forward-backward (FP64 and BF16 emulation)

Parity status of each function is stated in its docstring ("pinned by" or
"parity unpinned").
"""
