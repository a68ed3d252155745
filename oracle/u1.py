"""Oracle: the two-site variational fit with U(1)-symmetric tensors stored as dictionaries of
dense blocks (complex128). TEST INFRASTRUCTURE ONLY (see the package docstring).

Abelian symmetry as in the Heisenberg/XXZ example (Sec. 2.4; symmetric tensors, Sec. 1 and
Sec. 9): every leg index carries a charge and a tensor is nonzero only where the charges balance.
Conventions (shared with the device path and listed in the design notes):
  * physical index s has charge qp[s]; a bond's sector table is a dict {charge: dimension};
  * MPS site M[a][s][b] is nonzero only for q(b) = q(a) + qp[s]; it is stored as blocks
    {(q(a), s): array (dim q(a), dim q(a) + qp[s])}; the left end bond is {0: 1};
  * MPO site W[alpha][s'][s][beta] (dense, with level charges lc) is nonzero only for
    lc[alpha] + qp[s'] = qp[s] + lc[beta]; the MPO bond indices are grouped by charge class;
  * environments E[bra][mpo][ket] are nonzero only for q(bra) = q(ket) + lc[mpo]; stored as
    blocks {(q(bra), c): array (dim q(bra), #alpha of class c, dim q(bra) - c)}.
The fit follows the dense oracle (oracle.fit.fit_step) step for step; the only difference is the
truncation: the projected two-site tensor is block diagonal in the charge Q of the new bond, each
block is factorised by its own FP64 SVD and the singular values of all blocks compete for the D
kept ones (k = min(D, #{sigma > cutoff * sigma_max}) over all blocks, largest first).
"""
from __future__ import annotations

import numpy as np

_EINSUM = ("greedy", 2 ** 40)


def classes(lc):
    """{charge: array of MPO bond indices with that level charge} (ascending indices)."""
    lc = np.asarray(lc)
    return {int(c): np.flatnonzero(lc == c) for c in np.unique(lc)}


def check_blocks(site: dict, left: dict, right: dict, qp):
    for (qa, s), blk in site.items():
        qb = qa + int(qp[s])
        assert qa in left and qb in right and blk.shape == (left[qa], right[qb]), (qa, s, blk.shape)


def to_dense(sites, bonds, qp):
    """Dense MPS (indices of each bond in ascending charge order) from blocks and sector tables."""
    out = []
    for i, site in enumerate(sites):
        left, right = bonds[i], bonds[i + 1]
        lo = _offsets(left)
        ro = _offsets(right)
        M = np.zeros((sum(left.values()), len(qp), sum(right.values())), dtype=np.complex128)
        for (qa, s), blk in site.items():
            qb = qa + int(qp[s])
            M[lo[qa]:lo[qa] + left[qa], s, ro[qb]:ro[qb] + right[qb]] = blk
        out.append(M)
    return out


def from_dense(dense, bonds, qp):
    """Blocks of a dense MPS whose bond indices follow the sector tables in ascending charge."""
    sites = []
    for i, M in enumerate(dense):
        left, right = bonds[i], bonds[i + 1]
        lo, ro = _offsets(left), _offsets(right)
        site = {}
        for qa in left:
            for s in range(len(qp)):
                qb = qa + int(qp[s])
                if qb in right:
                    site[(qa, s)] = M[lo[qa]:lo[qa] + left[qa], s, ro[qb]:ro[qb] + right[qb]].copy()
        sites.append(site)
    return sites


def _offsets(table: dict) -> dict:
    out, o = {}, 0
    for q in sorted(table):
        out[q] = o
        o += table[q]
    return out


def boundary_env(lc, q0: int):
    """Env of a chain end: bra and ket bond {q0: 1}, the MPO on bond index 0."""
    cl = classes(lc)
    c = int(lc[0])
    E = np.zeros((1, len(cl[c]), 1), dtype=np.complex128)
    E[0, int(np.flatnonzero(cl[c] == 0)[0]), 0] = 1.0
    return {(q0 + c, c): E}


def env_left(Lenv, bra, W, lc, ket, qp):
    """L'[b', beta, b] = sum conj(bra[a', s', b']) L[a', alpha, a] W[alpha, s', s, beta] ket[a, s, b],
    block by block."""
    cl = classes(lc)
    out = {}
    for (qa_, c), E in Lenv.items():
        qa = qa_ - c
        for sp in range(len(qp)):
            Bb = bra.get((qa_, sp))
            if Bb is None:
                continue
            qb_ = qa_ + int(qp[sp])
            for s in range(len(qp)):
                Kb = ket.get((qa, s))
                if Kb is None:
                    continue
                qb = qa + int(qp[s])
                c2 = qb_ - qb
                if c2 not in cl:
                    continue
                Wc = W[np.ix_(cl[c], [sp], [s], cl[c2])][:, 0, 0, :]
                blk = np.einsum('xu,xay,ab,yv->ubv', Bb.conj(), E, Wc, Kb, optimize=_EINSUM)
                key = (qb_, c2)
                out[key] = out[key] + blk if key in out else blk
    return out


def env_right(Renv, bra, W, lc, ket, qp):
    """R'[a', alpha, a] = sum conj(bra[a', s', b']) W[alpha, s', s, beta] ket[a, s, b] R[b', beta, b],
    block by block."""
    cl = classes(lc)
    out = {}
    for (qb_, c2), E in Renv.items():
        qb = qb_ - c2
        for sp in range(len(qp)):
            qa_ = qb_ - int(qp[sp])
            Bb = bra.get((qa_, sp))
            if Bb is None:
                continue
            for s in range(len(qp)):
                qa = qb - int(qp[s])
                Kb = ket.get((qa, s))
                if Kb is None:
                    continue
                c = qa_ - qa
                if c not in cl:
                    continue
                Wc = W[np.ix_(cl[c], [sp], [s], cl[c2])][:, 0, 0, :]
                blk = np.einsum('xu,ab,yv,ubv->xay', Bb.conj(), Wc, Kb, E, optimize=_EINSUM)
                key = (qa_, c)
                out[key] = out[key] + blk if key in out else blk
    return out


def theta_blocks(Lenv, M1, W1, M2, W2, Renv, lc1, lc2, lc3, qp, left_bra: dict, right_bra: dict):
    """Projected two-site tensor Theta[a', s', t', c'] as blocks by the charge Q of the middle bond:
    {Q: array (rows (s', a') with q(a') = Q - qp[s'], concatenated over s'; columns (t', c') with
    q(c') = Q + qp[t'], concatenated over t')}; left_bra / right_bra: the sector tables of the outer
    bra bonds. The entry is the sum of L M1 W1 M2 W2 R over every index the definition sums."""
    d = len(qp)
    cl1, cl2, cl3 = classes(lc1), classes(lc2), classes(lc3)
    # left half: LB[(Q, s', c2, qb)] = array (dim a', n_c2, dim b)
    LB = {}
    for (qa_, c1), E in Lenv.items():
        qa = qa_ - c1
        for sp in range(d):
            Q = qa_ + int(qp[sp])
            for s in range(d):
                Kb = M1.get((qa, s))
                if Kb is None:
                    continue
                qb = qa + int(qp[s])
                c2 = Q - qb
                if c2 not in cl2:
                    continue
                Wc = W1[np.ix_(cl1[c1], [sp], [s], cl2[c2])][:, 0, 0, :]
                blk = np.einsum('xay,ab,yv->xbv', E, Wc, Kb, optimize=_EINSUM)
                key = (Q, sp, c2, qb)
                LB[key] = LB[key] + blk if key in LB else blk
    # right half: RB[(Q, t', c2, qb)] = array (n_c2, dim b, dim c')
    RB = {}
    for (qc_, c3), E in Renv.items():
        qc = qc_ - c3
        for tp in range(d):
            Q = qc_ - int(qp[tp])
            for t in range(d):
                qb = qc - int(qp[t])
                Kb = M2.get((qb, t))
                if Kb is None:
                    continue
                c2 = Q - qb
                if c2 not in cl2:
                    continue
                Wc = W2[np.ix_(cl2[c2], [tp], [t], cl3[c3])][:, 0, 0, :]
                blk = np.einsum('bg,yv,ugv->byu', Wc, Kb, E, optimize=_EINSUM)
                key = (Q, tp, c2, qb)
                RB[key] = RB[key] + blk if key in RB else blk
    out = {}
    for Q in sorted({k[0] for k in LB} & {k[0] for k in RB}):
        rows = [(sp, Q - int(qp[sp])) for sp in range(d) if Q - int(qp[sp]) in left_bra]
        cols = [(tp, Q + int(qp[tp])) for tp in range(d) if Q + int(qp[tp]) in right_bra]
        if not rows or not cols:
            continue
        R = sum(left_bra[qa] for _, qa in rows)
        C = sum(right_bra[qc] for _, qc in cols)
        T = np.zeros((R, C), dtype=np.complex128)
        r0 = 0
        for sp, qa in rows:
            c0 = 0
            for tp, qc in cols:
                acc = np.zeros((left_bra[qa], right_bra[qc]), dtype=np.complex128)
                for (Q_, sp_, c2, qb), A in LB.items():
                    if Q_ != Q or sp_ != sp:
                        continue
                    B = RB.get((Q, tp, c2, qb))
                    if B is not None:
                        acc += np.einsum('xbv,bvu->xu', A, B, optimize=_EINSUM)
                T[r0:r0 + left_bra[qa], c0:c0 + right_bra[qc]] = acc
                c0 += right_bra[qc]
            r0 += left_bra[qa]
        out[Q] = (T, rows, cols)
    return out


def truncate(blocks, Dmax: int, cutoff: float):
    """FP64 SVD of every charge block; the D largest singular values over all blocks are kept
    (k = min(D, #{sigma > cutoff * sigma_max}) >= 1, ties in favour of the lower charge, then the
    earlier value). Returns {Q: (U[:, :k_Q], S[:k_Q], Vh[:k_Q])} for k_Q > 0 and the discarded
    weight (sum of the dropped sigma^2 over the sum of all)."""
    fac, cand = {}, []
    for Q, (T, _, _) in blocks.items():
        U, S, Vh = np.linalg.svd(T, full_matrices=False)
        fac[Q] = (U, S, Vh)
        cand += [(-float(x), Q, j) for j, x in enumerate(S)]
    cand.sort()
    smax = -cand[0][0]
    n_above = sum(1 for x, _, _ in cand if -x > cutoff * smax) if smax > 0 else 1
    k = max(1, min(Dmax, n_above))
    keep = {}
    for _, Q, j in cand[:k]:
        keep[Q] = keep.get(Q, 0) + 1
    tot = sum(x * x for x, _, _ in cand)
    disc = sum(x * x for x, _, _ in cand[k:]) / tot if tot > 0 else 0.0
    out = {}
    for Q, kq in keep.items():
        U, S, Vh = fac[Q]
        out[Q] = (U[:, :kq], S[:kq], Vh[:kq])
    return out, disc


def right_canonicalize(sites, bonds, qp):
    """Right-canonical copy (QR of each site's adjoint per left-bond charge, last site to the
    second); returns (sites, bonds)."""
    sites = [dict(s) for s in sites]
    bonds = [dict(b) for b in bonds]
    d = len(qp)
    for i in range(len(sites) - 1, 0, -1):
        left, right = bonds[i], bonds[i + 1]
        new_left, Rs = {}, {}
        for qa in sorted(left):
            cols = [(s, qa + int(qp[s])) for s in range(d) if (qa, s) in sites[i]]
            if not cols:
                continue
            M = np.concatenate([sites[i][(qa, s)] for s, _ in cols], axis=1)  # (Da, sum Db)
            Qm, R = np.linalg.qr(M.conj().T)  # (sum Db, k), (k, Da)
            k = Qm.shape[1]
            new_left[qa] = k
            Rs[qa] = R
            c0 = 0
            for s, qb in cols:
                sites[i][(qa, s)] = Qm[c0:c0 + right[qb]].conj().T.copy()
                c0 += right[qb]
        for (qx, s), blk in list(sites[i - 1].items()):
            qa = qx + int(qp[s])
            if qa in Rs:
                sites[i - 1][(qx, s)] = blk @ Rs[qa].conj().T
            else:
                del sites[i - 1][(qx, s)]
        bonds[i] = new_left
    return sites, bonds


def fit_step(psi, bonds, W, lc, qp, Dmax: int, nsweeps: int = 2, cutoff: float = 1e-14):
    """One time step: the two-site variational fit of W|psi> with U(1) blocks (module docstring).
    psi: list of block dicts; bonds: L+1 sector tables; W: one dense MPO tensor (all sites) with
    level charges lc. Returns (phi, phi_bonds, stats) with stats = dict(norm, discarded)."""
    L = len(psi)
    phi, pb = right_canonicalize(psi, bonds, qp)
    Lenv = [None] * (L + 1)
    Renv = [None] * (L + 1)
    Lenv[0] = boundary_env(lc, next(iter(pb[0])))
    Renv[L] = boundary_env(lc, next(iter(pb[L])))
    for i in range(L - 1, 1, -1):
        Renv[i] = env_right(Renv[i + 1], phi[i], W, lc, psi[i], qp)
    d = len(qp)
    discarded, S = [], None
    for _ in range(nsweeps):
        for direction in (0, 1):
            order = range(0, L - 1) if direction == 0 else range(L - 2, -1, -1)
            for i in order:
                blocks = theta_blocks(Lenv[i], psi[i], W, psi[i + 1], W, Renv[i + 2], lc, lc, lc, qp,
                                      pb[i], pb[i + 2])
                kept, disc = truncate(blocks, Dmax, cutoff)
                discarded.append(disc)
                new_bond = {Q: kept[Q][1].size for Q in sorted(kept)}
                site_i, site_j = {}, {}
                for Q, (U, Sq, Vh) in kept.items():
                    _, rows, cols = blocks[Q]
                    A = U if direction == 0 else U * Sq[None, :]
                    B = (Sq[:, None] * Vh) if direction == 0 else Vh
                    r0 = 0
                    for sp, qa in rows:
                        site_i[(qa, sp)] = A[r0:r0 + pb[i][qa]].copy()
                        r0 += pb[i][qa]
                    c0 = 0
                    for tp, qc in cols:
                        site_j[(Q, tp)] = B[:, c0:c0 + pb[i + 2][qc]].copy()
                        c0 += pb[i + 2][qc]
                S = np.concatenate([kept[Q][1] for Q in kept])
                phi[i], phi[i + 1], pb[i + 1] = site_i, site_j, new_bond
                if direction == 0 and i < L - 2:
                    Lenv[i + 1] = env_left(Lenv[i], phi[i], W, lc, psi[i], qp)
                if direction == 1 and i > 0:
                    Renv[i + 1] = env_right(Renv[i + 2], phi[i + 1], W, lc, psi[i + 1], qp)
    norm = float(np.linalg.norm(S))
    if norm > 0:
        phi[0] = {k: v / norm for k, v in phi[0].items()}
    return phi, pb, dict(norm=norm, discarded=discarded)
