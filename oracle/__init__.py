"""Plain CPU oracle for higher-order MPO time evolution (complex128).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or link
anything in this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg use it. It shares no code with the device library.

Modules
  mpo    -- level bookkeeping, powers of the Hamiltonian MPO and the construction of
            the order-N time-evolution MPO (Sec. 2.5, Alg. 1, Alg. 2, Alg. 3, Alg. 4).
  fit    -- environments, projected two-site tensor, FP64 SVD truncation and the
            variational sweeping fit of W|psi> at fixed maximal bond dimension (Sec. 2.2):
            two-site and one-site, from a right-canonical or a zip-up guess; overlaps and
            MPO expectation values.
  u1     -- the two-site fit with U(1)-symmetric tensors stored as dictionaries of charge
            blocks (Sec. 2.4 XXZ example).
  dense  -- dense references for tiny chains: contracted operators, exact exponentials,
            MPS <-> state vectors.

Parity status: every function is pinned by a test that does not re-type its own
formula (printed tables, the bond-dimension table, error scaling, closed forms,
brute force). The order-(N+1) terms that the extension step (Alg. 3) adds are pinned
at every order N = 1..4 against a brute-force sum over products of Hamiltonian terms
(Sec. 5: every term of order N+1 whose N+1 actions overlap at most N times); the
compressions that follow it on the extended operator (Alg. 2, Alg. 4) are pinned by
the printed tables for N <= 2 and, for N >= 3, only through the bond-dimension
table, the error order, Alg. 2's exactness on the unextended operator and the
coefficient-wise exactness of the orders 0..N of the finished operator.
"""
