"""FP64 CPU oracle for the fermionic state-vector path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
anything in this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP library.

Three tiers, each written from the definitions (operators applied one at a
time on Jordan-Wigner qubit strings):

* ``dense``  (T1) -- literal 2^n complex128 state; every Hamiltonian term and
  every density-matrix element applied as an operator string.  n <= ~14.
* ``brute``  (T2) -- 2^n x 2^n sparse matrices from Kronecker products of
  Jordan-Wigner factors, rotations by matrix exponential, FCI by dense eigh.
  n <= ~10.  An independent route to every sign.
* ``sector`` (T3) -- C/OpenMP, only the (N_alpha, N_beta) sector stored;
  rotations, Hamiltonian, 1-RDM and the stored-state adjoint gradient.  n <= 30.

Every function states the passage of the paper it follows.
"""
