"""Plain FP64 CPU oracle for the CD/FNS IP-EOM-CCSD hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package;
only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code with the HIP library: it re-derives every quantity from
the paper's definitions in plain NumPy, complex128 throughout.

Modules
  integrals  antisymmetrised integrals from Cholesky vectors (Eq. 21-23)
  ccsd       CCSD amplitude equations (Eq. 12-15), Jacobi + DIIS
  eom        H-bar blocks, IP-EOM-CCSD sigma vectors (Eq. 16-18), dense eig, Davidson
  fns        MP2 virtual density and frozen natural spinors (Eq. 24-28)
  cd         single-step pivoted Cholesky of AO integrals and MO transform (Eq. 21-22)
  fockspace  brute-force second-quantised checks on tiny systems (FCI, e^-T H e^T)
  mlp        FP64 reference of the learned amplitude-update network

Every function without an independent pin says "parity unpinned"; the pins
live in tests/test_oracle_*.py.
"""
