"""Plain CPU oracle for higher-order MPO time evolution (complex128).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or link
anything in this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg use it. It shares no code with the device library.

Modules
  mpo    -- level bookkeeping, powers of the Hamiltonian MPO and the construction of
            the order-N time-evolution MPO (Sec. 2.5, Alg. 1, Alg. 2, Alg. 3, Alg. 4).
  fit    -- environments, projected two-site tensor, FP64 SVD truncation and the
            variational sweeping fit of W|psi> at fixed maximal bond dimension (Sec. 2.2).
  dense  -- dense references for tiny chains: contracted operators, exact exponentials,
            MPS <-> state vectors.

Parity status: every function is pinned by a test that does not re-type its own
formula (printed tables, the bond-dimension table, error scaling, closed forms,
brute force), except the order-(N+1) coefficients of the extended MPO for N >= 3,
which no printed table fixes ("parity partly unpinned": only the bond-dimension
table, the error-order test and the on-site closed form constrain them).
"""
