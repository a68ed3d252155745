"""Pin of the extension step (Sec. 5, Alg. 3) at every order, against a brute-force sum that
shares nothing with the level machinery of the oracle.

Sec. 5 states what the extension adds: to the order-N operator it adds every term of order N+1
in which the N+1 actions of the Hamiltonian overlap at most N times, i.e. every ordered product
h_1 h_2 ... h_{N+1} of Hamiltonian terms except those in which all N+1 terms stretch across one
common bond (the all-middle level (2,...,2) of H^{N+1}, which the order-N level set cannot hold),
each with the prefactor 1/(N+1)! of the exponential series. The terms h of a first-degree MPO
Hamiltonian (Sec. 2.3) are enumerated directly here: the on-site D_j, and for every interval
[i, j] the string C_i A_{i+1} ... A_{j-1} B_j summed over the middle-level indices.

With T_b the terms crossing bond b, the products of terms sharing a common bond are counted by
inclusion and exclusion over the (contiguous) set of commonly crossed bonds:
    sum_b (sum T_b)^{N+1} - sum_b (sum T_b & T_{b+1})^{N+1}.
The tau^k coefficients of the contracted operator l . W(tau) ... W(tau) . r are extracted exactly
(up to rounding) by a discrete Fourier transform over tau on the unit circle (the operator is a
polynomial in tau of degree below the number of sample points).

The extended operator is taken after the extension and the fold (Alg. 3, then Alg. 1): the later
compressions (Alg. 2 on the extended operator, Alg. 4) keep the orders up to N exact but are
free to change order N+1 (Sec. 6 states this for Alg. 4); they are pinned by the printed tables
of Sec. 5-6 and Appendix A for N <= 2, the bond-dimension table and the error-order tests.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import dense, mpo
from paper_2302_14181_amd import workloads as wl


def _kron(ops):
    out = np.eye(1, dtype=np.complex128)
    for o in ops:
        out = np.kron(out, o)
    return out


def _interval_terms(H, L):
    """{(i, j): dense operator of all Hamiltonian terms on the interval [i, j]}."""
    d, chi = H.d, H.chi
    eye = np.eye(d, dtype=np.complex128)
    terms = {}
    for j in range(L):
        ops = [eye] * L
        ops[j] = H.Dloc
        terms[(j, j)] = _kron(ops)
    for i in range(L):
        for j in range(i + 1, L):
            tot = np.zeros((d ** L, d ** L), dtype=np.complex128)
            for path in itertools.product(range(chi), repeat=j - i):
                ops = [eye] * L
                ops[i] = H.C[path[0]]
                for m in range(1, j - i):
                    ops[i + m] = H.A[path[m - 1], path[m]]
                ops[j] = H.B[path[-1]]
                tot += _kron(ops)
            terms[(i, j)] = tot
    return terms


def _brute_force(H, L, K):
    """(H, (1/K!) * sum of the K-fold ordered products of terms with no commonly crossed bond)."""
    terms = _interval_terms(H, L)
    Hs = sum(terms.values())
    total = np.linalg.matrix_power(Hs, K)
    for b in range(L - 1):  # bond between sites b and b + 1
        crossing = sum((t for (i, j), t in terms.items() if i <= b < j), np.zeros_like(Hs))
        total -= np.linalg.matrix_power(crossing, K)
        if b + 1 < L - 1:
            both = sum((t for (i, j), t in terms.items() if i <= b and j >= b + 2), np.zeros_like(Hs))
            total += np.linalg.matrix_power(both, K)
    return Hs, total / math.factorial(K)


def _extended_folded(H, N, tau):
    O = mpo.hamiltonian_power(H, N)
    O = mpo.extend(O, H, tau)
    O = mpo.fold(O, tau)
    W, _, _ = mpo.assemble(O)
    return W


def _taylor_coefficients(build, L, kmax, M=32):
    """tau^k coefficients, k = 0..kmax, of the dense operator l . W(tau)^L . r (l = r = e_0)."""
    F = np.array([dense.dense_evolution_mpo(build(np.exp(2j * np.pi * m / M)), L) for m in range(M)])
    return [np.tensordot(np.exp(-2j * np.pi * np.arange(M) * k / M) / M, F, axes=(0, 0))
            for k in range(kmax + 1)]


@pytest.mark.parametrize("N,chi", [(1, 1), (1, 2), (2, 1), (2, 2), (3, 1), (3, 2)])
def test_extension_adds_every_term_overlapping_at_most_N_times(N, chi):
    L = 4
    H = wl.random_blocks(np.random.default_rng(700 + 10 * N + chi), 2, chi)
    Hs, target = _brute_force(H, L, N + 1)
    Hd = dense.dense_hamiltonian(mpo.hamiltonian_mpo(H), L)
    np.testing.assert_allclose(Hs, Hd, atol=1e-13)  # the term enumeration is the Hamiltonian
    # the polynomial degree is at most L (N + 1) < M = 32 (fold weights tau^N, extension tau)
    c = _taylor_coefficients(lambda t: _extended_folded(H, N, t), L, N + 1)
    for k in range(N + 1):  # orders 0..N: the exponential series itself
        ref = np.linalg.matrix_power(Hd, k) / math.factorial(k)
        assert np.abs(c[k] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()), k
    scale = np.abs(target).max()
    assert np.abs(c[N + 1] - target).max() <= 1e-12 * scale
    # the excluded products are a sizeable part of the full order-(N+1) term (the pin is not vacuous)
    full = np.linalg.matrix_power(Hd, N + 1) / math.factorial(N + 1)
    assert np.abs(full - target).max() > 1e-3 * scale


@pytest.mark.slow
def test_extension_fourth_order():
    """N = 4 (chi = 1, L = 5): the highest order the builder supports."""
    N, L = 4, 5
    H = wl.random_blocks(np.random.default_rng(741), 2, 1)
    _, target = _brute_force(H, L, N + 1)
    c = _taylor_coefficients(lambda t: _extended_folded(H, N, t), L, N + 1, M=32)
    assert np.abs(c[N + 1] - target).max() <= 1e-12 * np.abs(target).max()


@pytest.mark.parametrize("variant", ["V1", "V2"])
@pytest.mark.parametrize("N,chi", [(1, 2), (2, 2), (3, 1), (3, 2), (4, 1)])
def test_orders_up_to_N_exact(N, chi, variant):
    """Every tau^k coefficient, k <= N, of the finished operator (all compressions applied) is
    H^k / k! exactly, coefficient by coefficient (a sharper form of the error law of Sec. 8.1)."""
    L = 4
    H = wl.random_blocks(np.random.default_rng(800 + 10 * N + chi), 2, chi)
    Hd = dense.dense_hamiltonian(mpo.hamiltonian_mpo(H), L)
    # per-site degree <= 2N + 1 (fold and Alg. 4 weights up to tau^N on extended blocks)
    M = 64 if L * (2 * N + 1) < 64 else 128
    c = _taylor_coefficients(lambda t: mpo.build_mpo(H, N, t, variant), L, N, M=M)
    for k in range(N + 1):
        ref = np.linalg.matrix_power(Hd, k) / math.factorial(k)
        assert np.abs(c[k] - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max()), k
