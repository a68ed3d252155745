"""Seeded synthetic inputs shared by the device path, the tests and the benchmark.

This module only *describes* inputs: the Jordan blocks (A, B, C, Dloc) of the
Hamiltonians used as workloads (Sec. 2.3 and the examples of Sec. 2.4 of the
paper), product states, and seeded random tensors. It contains none of the
method's arithmetic: no MPO construction, no contraction, no factorisation.

Conventions (all arrays numpy complex128, row-major):
  Dloc[s', s], C[k][s', s], B[k][s', s], A[k][l][s', s]  with k, l < chi.
  The Hamiltonian represented is  H = sum_i (Dloc_i + sum_k C_i^k B_{i+1}^k
  + sum_{k,l} C_i^k A_{i+1}^{kl} B_{i+2}^l + ...).
  MPS site tensors M[a][s][b] (left bond, physical, right bond).
"""
from __future__ import annotations

import dataclasses
import numpy as np

SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
ID2 = np.eye(2, dtype=np.complex128)


@dataclasses.dataclass
class JordanBlocks:
    """Blocks of a first-degree Hamiltonian MPO [[I, C, Dloc], [0, A, B], [0, 0, I]]."""
    A: np.ndarray  # (chi, chi, d, d)
    B: np.ndarray  # (chi, d, d)
    C: np.ndarray  # (chi, d, d)
    Dloc: np.ndarray  # (d, d)
    inner_charge: np.ndarray | None = None  # (chi,) U(1) charge carried by the middle level
    phys_charge: np.ndarray | None = None  # (d,)

    @property
    def d(self) -> int:
        return self.Dloc.shape[0]

    @property
    def chi(self) -> int:
        return self.B.shape[0]


def tfim(g: float, J: float = 1.0) -> JordanBlocks:
    """Transverse-field Ising chain H = -J sum Z_i Z_{i+1} - g sum X_i (chi = 1)."""
    return JordanBlocks(
        A=np.zeros((1, 1, 2, 2), dtype=np.complex128),
        B=SZ[None].copy(),
        C=(-J * SZ)[None].copy(),
        Dloc=(-g * SX).copy(),
    )


def tfim_cylinder(Ly: int, h: float, J: float = 1.0) -> JordanBlocks:
    """Transverse-field Ising model on a cylinder of circumference Ly with spiral boundary
    conditions, as a chain along the spiral (Sec. 2.3, the cylinder example):
    H = -J sum (Z_i Z_{i+1} + Z_i Z_{i+Ly}) + h sum X_i.
    The middle level is a shift register of Ly steps (chi = Ly): a Z placed r sites back sits in
    register r - 1 and closes at distance 1 or Ly."""
    A = np.zeros((Ly, Ly, 2, 2), dtype=np.complex128)
    for j in range(Ly - 1):
        A[j, j + 1] = ID2
    C = np.zeros((Ly, 2, 2), dtype=np.complex128)
    C[0] = -J * SZ
    B = np.zeros((Ly, 2, 2), dtype=np.complex128)
    B[0] += SZ
    B[Ly - 1] += SZ  # (Ly = 1: both couplings close at distance 1)
    return JordanBlocks(A=A, B=B, C=C, Dloc=h * SX)


def lr_ising(coeffs, lambdas, g: float) -> JordanBlocks:
    """Ising chain with couplings J(r) = sum_k c_k lambda_k^(r-1) plus transverse field.

    H = -sum_{i<j} J(j-i) Z_i Z_j - g sum X_i, one middle level per exponential.
    """
    K = len(coeffs)
    A = np.zeros((K, K, 2, 2), dtype=np.complex128)
    for k in range(K):
        A[k, k] = lambdas[k] * ID2
    C = np.stack([-coeffs[k] * SZ for k in range(K)])
    B = np.stack([SZ for _ in range(K)])
    return JordanBlocks(A=A, B=B, C=C, Dloc=-g * SX)


def xxz(delta: float) -> JordanBlocks:
    """Spin-1/2 XXZ chain H = sum (Sx Sx + Sy Sy + delta Sz Sz), S = sigma/2 (chi = 3).

    Written with S+ S- terms so that each middle level carries a definite U(1)
    charge (number of up spins): C = (S+/2, S-/2, delta Sz), B = (S-, S+, Sz).
    Physical basis order: index 0 = up (charge 1), index 1 = down (charge 0).
    """
    sp = np.array([[0, 1], [0, 0]], dtype=np.complex128)
    sm = sp.T.copy()
    sz = 0.5 * SZ
    C = np.stack([0.5 * sp, 0.5 * sm, delta * sz])
    B = np.stack([sm, sp, sz])
    A = np.zeros((3, 3, 2, 2), dtype=np.complex128)
    return JordanBlocks(A=A, B=B, C=C, Dloc=np.zeros((2, 2), dtype=np.complex128),
                        inner_charge=np.array([1, -1, 0]), phys_charge=np.array([1, 0]))


def random_blocks(rng: np.random.Generator, d: int, chi: int, a_scale: float = 0.5) -> JordanBlocks:
    """Generic non-Hermitian blocks with complex-normal entries; A scaled to spectral radius < 1."""
    def cn(*shape):
        return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)
    A = cn(chi, chi, d, d) * (a_scale / max(1.0, np.sqrt(chi * d)))
    return JordanBlocks(A=A, B=cn(chi, d, d), C=cn(chi, d, d), Dloc=cn(d, d))


def random_hermitian_blocks(rng: np.random.Generator, d: int, chi: int, a_scale: float = 0.5) -> JordanBlocks:
    """Blocks of a Hermitian Hamiltonian with chi exponentially decaying couplings:
    C^k = c_k O_k, B^k = O_k, A^{kl} = lambda_k delta_{kl} I with Hermitian O_k, Dloc and real
    c_k, lambda_k (|lambda_k| < 1), i.e. H = sum_i h_i + sum_{i<j,k} c_k lambda_k^(j-i-1) O_k^i O_k^j."""
    def herm():
        x = complex_normal(rng, (d, d))
        return 0.5 * (x + x.conj().T)
    ops = np.stack([herm() for _ in range(chi)])
    c = rng.uniform(-1.0, 1.0, size=chi)
    lam = a_scale * rng.uniform(0.2, 1.0, size=chi)
    A = np.zeros((chi, chi, d, d), dtype=np.complex128)
    for k in range(chi):
        A[k, k] = lam[k] * np.eye(d)
    return JordanBlocks(A=A, B=ops.copy(), C=c[:, None, None] * ops, Dloc=herm())


def product_state(L: int, local: np.ndarray) -> list[np.ndarray]:
    """Product MPS with every site in the normalised local state `local` (length d)."""
    v = np.asarray(local, dtype=np.complex128)
    v = v / np.linalg.norm(v)
    return [v.reshape(1, -1, 1).copy() for _ in range(L)]


def all_up(L: int, d: int = 2) -> list[np.ndarray]:
    e = np.zeros(d, dtype=np.complex128)
    e[0] = 1.0
    return product_state(L, e)


def infinite_temperature(L: int, d: int = 2) -> list[np.ndarray]:
    """Purified chain at beta = 0: on every site the normalised maximally entangled pair of a
    physical and an ancilla leg, sum_s |s>|s> / sqrt(d), local index s d + a (bond 1)."""
    local = np.zeros(d * d, dtype=np.complex128)
    local[[s * d + s for s in range(d)]] = 1 / np.sqrt(d)
    return [local.reshape(1, d * d, 1).copy() for _ in range(L)]


def bond_dims(L: int, d: int, D: int) -> list[int]:
    """Largest useful bond dimensions of an open chain capped at D: min(D, d^i, d^(L-i))."""
    out = []
    for i in range(L + 1):
        out.append(int(min(D, d ** min(i, L - i))))
    return out


def random_mps(rng: np.random.Generator, L: int, d: int, D: int, dims: list[int] | None = None) -> list[np.ndarray]:
    """MPS with seeded complex-normal site tensors (entries (x + i y)/sqrt(2)), bonds `dims`.

    Entries are scaled by 1/sqrt(d * D_right) so contractions stay O(1); the state is not
    normalised or canonicalised here.
    """
    if dims is None:
        dims = bond_dims(L, d, D)
    out = []
    for i in range(L):
        shape = (dims[i], d, dims[i + 1])
        x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)
        out.append(x / np.sqrt(d * dims[i + 1]))
    return out


def complex_normal(rng: np.random.Generator, shape) -> np.ndarray:
    """Entries (x + i y)/sqrt(2) with x, y ~ N(0, 1), drawn as one real block then one imaginary."""
    x = rng.standard_normal(shape)
    y = rng.standard_normal(shape)
    return (x + 1j * y) / np.sqrt(2)


def env_microbench_inputs(seed: int = 0, D: int = 256, d: int = 2, w: int = 8):
    """Seeded complex-normal operands of one environment update: E (D, w, D), ket M (D, d, D),
    bra N (D, d, D) and W (w, d, d, w), drawn in that order."""
    rng = np.random.default_rng(seed)
    E = complex_normal(rng, (D, w, D))
    M = complex_normal(rng, (D, d, D))
    N = complex_normal(rng, (D, d, D))
    W = complex_normal(rng, (w, d, d, w))
    return E, M, N, W


def batched_tfim_chains(seed: int = 2, n: int = 64):
    """The independent-chain batch: per chain (g, L, D) with g ~ U(0.5, 1.5), L drawn from
    {32, 64, 96, 128} and D from {32, 64, 128, 256}, uniformly and independently, drawn per chain
    in that order from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        g = float(rng.uniform(0.5, 1.5))
        L = int(rng.choice([32, 64, 96, 128]))
        D = int(rng.choice([32, 64, 128, 256]))
        out.append((g, L, D))
    return out


def u1_sector_tables(L: int, n_up: int, D: int, nsec: int = 15, seed: int = 1, width: float = 3.0):
    """Sector tables {charge: dimension} of the L + 1 bonds of a U(1) MPS with n_up up spins
    (charge = number of up spins to the left of the bond): on bond b the nsec charges nearest the
    mean filling b n_up / L that the chain can reach, with dimensions proportional to
    exp(-(q - qbar)^2 / (2 width^2)) (1 + 0.2 xi), xi ~ N(0, 1) from `seed`, rounded by largest
    remainder to a total of at most D, each at least 1 and at most the exact sector dimension
    min(C(b, q), C(L - b, n_up - q)). Bonds 0 and L are {0: 1} and {n_up: 1}."""
    from math import comb
    rng = np.random.default_rng(seed)
    tables = [{0: 1}]
    for b in range(1, L):
        lo, hi = max(0, n_up - (L - b)), min(b, n_up)
        qbar = b * n_up / L
        qs = sorted(range(lo, hi + 1), key=lambda q: (abs(q - qbar), q))[:nsec]
        qs.sort()
        exact = {q: min(comb(b, q), comb(L - b, n_up - q)) for q in qs}
        wgt = np.array([np.exp(-(q - qbar) ** 2 / (2 * width ** 2)) * max(0.05, 1 + 0.2 * rng.standard_normal())
                        for q in qs])
        total = min(D, sum(exact.values()))
        raw = wgt / wgt.sum() * total
        dims = {q: max(1, min(exact[q], int(np.floor(r)))) for q, r in zip(qs, raw)}
        rem = sorted(zip(qs, raw - np.floor(raw)), key=lambda t: -t[1])
        while sum(dims.values()) < total:
            grown = False
            for q, _ in rem:
                if sum(dims.values()) >= total:
                    break
                if dims[q] < exact[q]:
                    dims[q] += 1
                    grown = True
            if not grown:
                break
        while sum(dims.values()) > total:
            q = max(dims, key=lambda x: dims[x])
            dims[q] -= 1
        tables.append({q: d for q, d in dims.items() if d > 0})
    tables.append({n_up: 1})
    return tables


def random_u1_mps(rng: np.random.Generator, tables, phys_charge):
    """Random U(1) MPS as blocks {(q_left, s): array (dim q_left, dim q_left + phys_charge[s])}
    with complex-normal entries, blocks only where both charges exist; the entries of a left index
    of charge q are scaled by 1 / sqrt(its number of entries, sum_s dim(q + phys_charge[s])), so
    that every row has unit expected norm and the state's norm stays of order one on long chains.
    Returns the list of site dicts."""
    d = len(phys_charge)
    sites = []
    for i in range(len(tables) - 1):
        left, right = tables[i], tables[i + 1]
        site = {}
        for qa, da in left.items():
            nrow = sum(right.get(qa + int(phys_charge[s]), 0) for s in range(d))
            for s in range(d):
                qb = qa + int(phys_charge[s])
                if qb in right:
                    site[(qa, s)] = complex_normal(rng, (da, right[qb])) / np.sqrt(nrow)
        sites.append(site)
    return sites


def u1_dense(sites, tables, phys_charge):
    """A U(1) MPS given as blocks laid out densely with every bond's indices in ascending charge:
    (list of (D_left, d, D_right) arrays, list of L + 1 per-index charge lists)."""
    d = len(phys_charge)
    out, charges = [], []
    for b, t in enumerate(tables):
        charges.append([q for q in sorted(t) for _ in range(t[q])])
    for i, site in enumerate(sites):
        left, right = tables[i], tables[i + 1]
        lo, ro, o = {}, {}, 0
        for q in sorted(left):
            lo[q] = o
            o += left[q]
        o = 0
        for q in sorted(right):
            ro[q] = o
            o += right[q]
        M = np.zeros((sum(left.values()), d, sum(right.values())), dtype=np.complex128)
        for (qa, s), blk in site.items():
            qb = qa + int(phys_charge[s])
            M[lo[qa]:lo[qa] + left[qa], s, ro[qb]:ro[qb] + right[qb]] = blk
        out.append(M)
    return out, charges
