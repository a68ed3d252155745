"""Oracle: order-N MPO approximation of exp(tau H) (complex128, plain Python + numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The Hamiltonian is a first-degree MPO in Jordan form with levels 1, 2, 3
(Sec. 2.3, eq. jordan_mpo):  H[1,1] = I, H[1,2] = C, H[1,3] = Dloc, H[2,2] = A,
H[2,3] = B, H[3,3] = I, all other blocks zero.  Level 2 carries a virtual index of
dimension chi, levels 1 and 3 are one-dimensional.

A block of an operator-valued level matrix is stored as a tensor of shape
(vdim(row level), d, d, vdim(column level)), indices [alpha, s_out, s_in, beta].

Readings of the paper used here (each is also listed with its reason in the design notes):
  * Powers (Sec. 2.5): the block of H^N between level tuples a and b is the operator
    product H[a_1,b_1] H[a_2,b_2] ... H[a_N,b_N] with copy 1 leftmost, and the
    Kronecker product of the virtual indices of the copies in position order.
  * Alg. 3 (extension) runs on the raw H^N, before the fold of Alg. 1; it visits target
    levels b that contain NO 1 (the printed condition "1 in b" would double-count the
    identity path), and n_1 / n_3 count the 1s of a_e and the 3s of b_e.
  * Alg. 1 (fold) processes a = 1..N in increasing order and removes each folded level at once.
  * Alg. 2 (exact compression) moves the 1s to the front (row merge) when n_3 <= n_1, and the
    3s to the BACK (column merge) otherwise, both stably, visiting levels lexicographically;
    the worked second-order example keeps (2,3) and removes (3,2).
  * Alg. 4 (approximate compression) visits levels with no 1 and at least one 3; it folds the
    column into the level obtained by replacing the 3s with 1s, in its Alg. 2 representative
    form (1s in front), with weight tau^k (N-k)!/N!, k = number of 3s.
  * Final level order: (1,...,1) first, then lexicographic; boundary vectors select (1,...,1)
    on both ends (Sec. 3, eq. boundary).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def all_levels(N: int) -> list[tuple[int, ...]]:
    """All level tuples {1,2,3}^N in lexicographic order (1 < 2 < 3)."""
    return [tuple(t) for t in itertools.product((1, 2, 3), repeat=N)]


def vdim(level: tuple[int, ...], chi: int) -> int:
    """Virtual dimension of a level tuple: chi per entry equal to 2 (Sec. 2.5)."""
    return chi ** sum(1 for x in level if x == 2)


def single_block(H, a: int, b: int):
    """Block H[a, b] of the Jordan-form Hamiltonian MPO as a (va, d, d, vb) tensor, or None."""
    d = H.Dloc.shape[0]
    if (a, b) in ((1, 1), (3, 3)):
        return np.eye(d, dtype=np.complex128).reshape(1, d, d, 1)
    if (a, b) == (1, 2):  # C[k][s', s] -> [0, s', s, k]
        return np.transpose(np.asarray(H.C, dtype=np.complex128), (1, 2, 0))[None]
    if (a, b) == (1, 3):
        return np.asarray(H.Dloc, dtype=np.complex128)[None, :, :, None]
    if (a, b) == (2, 2):  # A[k][l][s', s] -> [k, s', s, l]
        return np.transpose(np.asarray(H.A, dtype=np.complex128), (0, 2, 3, 1))
    if (a, b) == (2, 3):  # B[k][s', s] -> [k, s', s, 0]
        return np.asarray(H.B, dtype=np.complex128)[..., None]
    return None


def power_block(H, a: tuple[int, ...], b: tuple[int, ...]):
    """Block of H^N between level tuples a and b (Sec. 2.5): operator product on the physical
    legs (copy 1 leftmost), direct product on the virtual legs. None if structurally zero."""
    out = None
    for aj, bj in zip(a, b):
        blk = single_block(H, aj, bj)
        if blk is None:
            return None
        if out is None:
            out = blk
            continue
        va, d, _, vb = out.shape
        ua, _, _, ub = blk.shape
        # out[v, s', x, w] * blk[u, x, s, z] -> [v, u, s', s, w, z]
        t = np.einsum('vpxw,uxsz->vupswz', out, blk)
        out = t.reshape(va * ua, d, d, vb * ub)
    return out


class LevelMatrix:
    """Operator-valued block matrix over a set of present level tuples."""

    def __init__(self, N: int, chi: int, d: int):
        self.N, self.chi, self.d = N, chi, d
        self.levels: list[tuple[int, ...]] = []
        self.blocks: dict[tuple, np.ndarray] = {}

    def get(self, a, b):
        return self.blocks.get((a, b))

    def add(self, a, b, blk):
        if blk is None:
            return
        cur = self.blocks.get((a, b))
        self.blocks[(a, b)] = blk.copy() if cur is None else cur + blk

    def remove(self, c):
        self.levels.remove(c)
        for key in [k for k in self.blocks if k[0] == c or k[1] == c]:
            del self.blocks[key]

    def copy(self):
        o = LevelMatrix(self.N, self.chi, self.d)
        o.levels = list(self.levels)
        o.blocks = {k: v.copy() for k, v in self.blocks.items()}
        return o


def hamiltonian_power(H, N: int) -> LevelMatrix:
    """H^N as a level matrix over {1,2,3}^N (Sec. 2.5)."""
    d, chi = H.Dloc.shape[0], H.B.shape[0]
    O = LevelMatrix(N, chi, d)
    O.levels = all_levels(N)
    for a in O.levels:
        for b in O.levels:
            if all(x <= y for x, y in zip(a, b)):
                blk = power_block(H, a, b)
                if blk is not None:
                    O.blocks[(a, b)] = blk
    return O


def extend(O: LevelMatrix, H, tau: complex) -> LevelMatrix:
    """Alg. 3 (extension step, Sec. 5) applied to the raw H^N.

    For a source level a (skipped when it has no 2 but some 3) and a target level b with no 1,
    add  tau * N! / ((N+1)! n1 n3) * H^{N+1}[a_e, b_e]  for every position c where a 1 is inserted
    into a (giving a_e) and every position e where a 3 is inserted into b (giving b_e).
    """
    N = O.N
    out = O.copy()
    coef0 = tau * math.factorial(N) / math.factorial(N + 1)
    for a in O.levels:
        if 2 not in a and 3 in a:
            continue
        for b in O.levels:
            if 1 in b:
                continue
            acc = None
            for c in range(N + 1):
                ae = a[:c] + (1,) + a[c:]
                n1 = ae.count(1)
                for e in range(N + 1):
                    be = b[:e] + (3,) + b[e:]
                    n3 = be.count(3)
                    blk = power_block(H, ae, be)
                    if blk is None:
                        continue
                    term = (coef0 / (n1 * n3)) * blk
                    acc = term if acc is None else acc + term
            out.add(a, b, acc)
    return out


def fold(O: LevelMatrix, tau: complex) -> LevelMatrix:
    """Alg. 1 (Sec. 3): for k = 1..N, every level made of (N-k) 1s and k 3s is folded into the
    column of (1,...,1) with weight tau^k (N-k)!/N!, then its row and column are removed."""
    N = O.N
    out = O.copy()
    one = (1,) * N
    for k in range(1, N + 1):
        targets = [b for b in all_levels(N) if set(b) <= {1, 3} and b.count(3) == k]
        w = tau ** k * math.factorial(N - k) / math.factorial(N)
        for b in targets:
            if b not in out.levels:
                continue
            for r in list(out.levels):
                blk = out.get(r, b)
                if blk is not None:
                    out.add(r, one, w * blk)
            out.remove(b)
    return out


def ones_front(c: tuple[int, ...]) -> tuple[int, ...]:
    """Stable sort moving every 1 to the front (the other entries keep their order)."""
    return tuple(x for x in c if x == 1) + tuple(x for x in c if x != 1)


def threes_back(c: tuple[int, ...]) -> tuple[int, ...]:
    """Stable sort moving every 3 to the back."""
    return tuple(x for x in c if x != 3) + tuple(x for x in c if x == 3)


def exact_compress(O: LevelMatrix) -> LevelMatrix:
    """Alg. 2 (Sec. 4): merge levels with identical left (row merge) or right (column merge)
    environments, visiting the present levels in lexicographic order."""
    out = O.copy()
    for c in sorted(out.levels):
        if c not in out.levels:
            continue
        n1, n3 = c.count(1), c.count(3)
        if n3 <= n1:
            s = ones_front(c)
            if s != c:
                for col in list(out.levels):
                    out.add(s, col, out.get(c, col))
                out.remove(c)
        else:
            s = threes_back(c)
            if s != c:
                for row in list(out.levels):
                    out.add(row, s, out.get(row, c))
                out.remove(c)
    return out


def approx_compress(O: LevelMatrix, tau: complex) -> LevelMatrix:
    """Alg. 4 (Sec. 6): a level a with no 1 and k >= 1 threes is folded, with weight
    tau^k (N-k)!/N!, into the column of the level obtained by turning its 3s into 1s (written
    with its 1s in front), and removed."""
    N = O.N
    out = O.copy()
    for a in sorted(out.levels):
        if a not in out.levels or 1 in a or 3 not in a:
            continue
        k = a.count(3)
        b = ones_front(tuple(1 if x == 3 else x for x in a))
        if b not in out.levels:
            raise RuntimeError(f"approximate compression target {b} missing")
        w = tau ** k * math.factorial(N - k) / math.factorial(N)
        for r in list(out.levels):
            blk = out.get(r, a)
            if blk is not None:
                out.add(r, b, w * blk)
        out.remove(a)
    return out


def ordered_levels(O: LevelMatrix) -> list[tuple[int, ...]]:
    one = (1,) * O.N
    return [one] + sorted(l for l in O.levels if l != one)


def assemble(O: LevelMatrix):
    """Dense MPO tensor W[alpha, s', s, beta] with (1,...,1) at index 0, plus level offsets."""
    order = ordered_levels(O)
    offs, w = {}, 0
    for l in order:
        offs[l] = w
        w += vdim(l, O.chi)
    W = np.zeros((w, O.d, O.d, w), dtype=np.complex128)
    for (a, b), blk in O.blocks.items():
        W[offs[a]:offs[a] + blk.shape[0], :, :, offs[b]:offs[b] + blk.shape[3]] += blk
    return W, order, offs


def build_levels(H, N: int, tau: complex, variant: str = "V2") -> LevelMatrix:
    """Level matrix of the order-N time-evolution MPO.
    V1: Alg. 1 then Alg. 2.  V2: Alg. 3 (on H^N), Alg. 1, Alg. 2, then Alg. 4."""
    if N < 1:
        raise ValueError("order must be >= 1")
    O = hamiltonian_power(H, N)
    if variant == "V2":
        O = extend(O, H, tau)
    elif variant != "V1":
        raise ValueError(variant)
    O = fold(O, tau)
    O = exact_compress(O)
    if variant == "V2":
        O = approx_compress(O, tau)
    return O


def build_mpo(H, N: int, tau: complex, variant: str = "V2") -> np.ndarray:
    """Order-N MPO tensor W[alpha, s', s, beta] for exp(tau H); boundaries l = r = e_0."""
    W, _, _ = assemble(build_levels(H, N, tau, variant))
    return W


def level_charges(H, N: int, tau: complex, variant: str = "V2") -> np.ndarray:
    """U(1) charge of every MPO bond index: the sum of the middle-level charges at the
    2-positions of its level tuple (Kronecker order of the virtual indices)."""
    O = build_levels(H, N, tau, variant)
    q = np.asarray(H.inner_charge)
    out = []
    for l in ordered_levels(O):
        k = l.count(2)
        for idx in itertools.product(range(O.chi), repeat=k):
            out.append(int(sum(q[i] for i in idx)))
    return np.array(out, dtype=np.int64)


def hamiltonian_mpo(H) -> np.ndarray:
    """The Hamiltonian itself as an MPO tensor over levels (1, 2, 3): bond 1 + chi + 1.
    Boundaries: left selects level 1 (index 0), right selects level 3 (index chi + 1)."""
    d, chi = H.Dloc.shape[0], H.B.shape[0]
    w = chi + 2
    W = np.zeros((w, d, d, w), dtype=np.complex128)
    W[0, :, :, 0] = np.eye(d)
    W[w - 1, :, :, w - 1] = np.eye(d)
    W[0, :, :, 1:1 + chi] = np.transpose(H.C, (1, 2, 0))
    W[0, :, :, w - 1] = H.Dloc
    W[1:1 + chi, :, :, 1:1 + chi] = np.transpose(H.A, (0, 2, 3, 1))
    W[1:1 + chi, :, :, w - 1] = H.B
    return W


# Splitting composites (Sec. 8.3, splitting schemes): two first-order operators at the complex
# steps t1 tau and t2 tau, t1,2 = (1 +- i)/2, multiply to an operator accurate to second order
# (t1 + t2 = 1 and t1 t2 = 1/2 reproduce the tau and tau^2 / 2 terms of the exponential).
SPLIT_T1 = (1 + 1j) / 2
SPLIT_T2 = (1 - 1j) / 2


def compose(Wa: np.ndarray, Wb: np.ndarray) -> np.ndarray:
    """Site tensor of the operator product O_a O_b of two MPOs (O_b acts first):
    W[(alpha_a, alpha_b), s', s, (beta_a, beta_b)] = sum_m Wa[alpha_a, s', m, beta_a] Wb[alpha_b, m, s, beta_b];
    the bond is the Kronecker product of the two (boundary index 0 of both is index 0)."""
    wa, d, _, wa_r = Wa.shape
    wb, wb_r = Wb.shape[0], Wb.shape[3]
    X = np.einsum('apmb,cmsd->acpsbd', Wa, Wb)
    return X.reshape(wa * wb, d, d, wa_r * wb_r)


def split_composite(H, tau: complex, variant: str = "V2") -> np.ndarray:
    """O1(t1 tau) O1(t2 tau) as one MPO tensor (bond (1 + chi)^2 for V2)."""
    return compose(build_mpo(H, 1, SPLIT_T1 * tau, variant), build_mpo(H, 1, SPLIT_T2 * tau, variant))


# Finite temperature on a finite chain by purification: each site carries a physical and an
# ancilla leg, combined as s d + a (ancilla fastest); exp(-beta H / 2) acting on the physical legs
# of the product of maximally entangled pairs gives a state whose expectation values are thermal
# averages at inverse temperature beta (the finite-chain counterpart of the density matrix
# exp(-beta H) built in Sec. 8.4 for the thermodynamic limit).
def purify(W: np.ndarray) -> np.ndarray:
    """Site tensor of O (x) I: W'[alpha, (s', a'), (s, a), beta] = W[alpha, s', s, beta] delta(a', a)."""
    w, d, _, w2 = W.shape
    return np.einsum('apqb,xy->apxqyb', W, np.eye(d)).reshape(w, d * d, d * d, w2)
