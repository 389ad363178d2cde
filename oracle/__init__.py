"""FP64 CPU oracle for the two-site DMRG sigma-vector path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path never
calls it, and it shares no code with the HIP library or its Python binding.

Modules:
  fock      -- determinant basis, creation/annihilation operators, the ab initio
               Hamiltonian in a particle-number / spin sector, FCI energies
               (Sec. II.A.1).
  holstein  -- the Hubbard-Holstein model of Listing 1 (paper's printed energy).
  mps       -- MPS -> Fock-space embedding P and H_eff := P^T H P (the plain
               definition of the effective Hamiltonian of the two-site sweep,
               Sec. II.A.2).
  contract  -- the renormalised-operator contraction sigma = sum L W W R psi,
               environment updates and diag(H_eff), written as single einsum
               definitions on dense zero-padded arrays, plus a row-sampled form
               for full-size checks.
  davidson  -- one textbook Davidson step (Davidson 1975), the eigensolver the
               paper's sweeps use (Listing 1 passes its iteration cap).
"""
