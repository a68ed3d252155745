"""Oracle: variational two-site fit of W|psi> at bounded bond dimension (complex128).

TEST INFRASTRUCTURE ONLY (see the package docstring).

One time step (Sec. 2.2, Table 1 "(i)DMRG" row; Sec. 8.2: a variational sweeping optimisation
of the time-evolved MPS in every step): find the MPS phi with bonds <= Dmax that maximises
|<phi|W psi>|.  Readings of the paper (which leaves the details open), shared with the device
path and listed in the design notes:
  * guess phi = psi, brought to right-canonical form by QR from the last site to the second;
  * a sweep is a left-to-right pass over the bonds (0,1) .. (L-2,L-1) followed by a
    right-to-left pass over the same bonds; two sweeps per time step;
  * at every bond the exact projection Theta of W|psi> onto the current left/right bases is
    split by an SVD in FP64; k = min(Dmax, #{sigma_i > cutoff * sigma_1}) values are kept
    (k >= 1); left-to-right: phi_i = U, phi_{i+1} = S V^dag; right-to-left: phi_i = U S,
    phi_{i+1} = V^dag;
  * after the last visit phi is normalised; the norm before normalisation is |<phi_hat|W psi>|.

Tensor conventions: MPS site M[a, s, b]; MPO site W[alpha, s_out, s_in, beta]; environments
E[bra, mpo, ket].  The bra is conjugated inside the environment contractions.
"""
from __future__ import annotations

import numpy as np


# numpy's default einsum planner allows no intermediate larger than the largest operand, which
# for these networks leaves a single many-operand step that never reaches BLAS; the greedy
# planner with room for pairwise intermediates evaluates the same expression through BLAS.
_EINSUM = ("greedy", 2 ** 40)


def env_left(Lenv, bra, W, ket):
    """L'[b', beta, b] = sum conj(bra[a', s', b']) L[a', alpha, a] W[alpha, s', s, beta] ket[a, s, b]."""
    return np.einsum('xay,xpu,apsb,ysv->ubv', Lenv, bra.conj(), W, ket, optimize=_EINSUM)


def env_right(Renv, bra, W, ket):
    """R'[a', alpha, a] = sum conj(bra[a', s', b']) W[alpha, s', s, beta] ket[a, s, b] R[b', beta, b]."""
    return np.einsum('xpu,apsb,ysv,ubv->xay', bra.conj(), W, ket, Renv, optimize=_EINSUM)


def theta_two_site(Lenv, M1, W1, M2, W2, Renv):
    """Projected two-site tensor Theta[a', s', t', c'] =
    sum L[a', alpha, a] M1[a, s, b] W1[alpha, s', s, beta] M2[b, t, c] W2[beta, t', t, gamma] R[c', gamma, c]."""
    return np.einsum('xay,ysb,apsg,btc,gqtz,uzc->xpqu', Lenv, M1, W1, M2, W2, Renv, optimize=_EINSUM)


def svd_truncate(mat, Dmax: int, cutoff: float):
    """FP64 SVD of a matrix, keeping k = min(Dmax, #{sigma > cutoff * sigma_1}) >= 1 values.
    Returns U[:, :k], S[:k], Vh[:k], and the discarded weight sum_{i>=k} sigma_i^2 / sum sigma_i^2."""
    U, S, Vh = np.linalg.svd(mat, full_matrices=False)
    if S.size == 0:
        raise ValueError("empty matrix")
    if S[0] > 0:
        k = int(np.count_nonzero(S > cutoff * S[0]))
    else:
        k = 1
    k = max(1, min(Dmax, k))
    tot = float(np.sum(S ** 2))
    disc = float(np.sum(S[k:] ** 2)) / tot if tot > 0 else 0.0
    return U[:, :k], S[:k], Vh[:k], disc


def right_canonicalize(ms):
    """Right-canonical copy of an MPS: QR of each site's adjoint from the last site to the second;
    the triangular factor is absorbed into the site on the left. Bond i becomes
    min(D_left, d * D_right) where that is smaller."""
    out = [m.copy() for m in ms]
    for i in range(len(out) - 1, 0, -1):
        a, d, b = out[i].shape
        Q, R = np.linalg.qr(out[i].reshape(a, d * b).conj().T)  # (d b) x k, k x a
        k = Q.shape[1]
        out[i] = Q.conj().T.reshape(k, d, b)
        out[i - 1] = np.einsum('xsa,ka->xsk', out[i - 1], R.conj())
    return out


def boundary_env(w: int):
    E = np.zeros((1, w, 1), dtype=np.complex128)
    E[0, 0, 0] = 1.0
    return E


def zipup_guess(psi, Ws, Dmax: int, cutoff: float = 1e-14):
    """Zip-up application of W to psi (Sec. 2.2, Table 1 zip-up row): W|psi> compressed site by
    site with SVDs, without bringing psi into canonical form first. Readings (the paper only
    names the method): the zip runs from the right end to the left, so that its sites come out
    right-orthonormal, as the two-site fit wants its guess. A carry C[k, beta, b] (k: the new bond
    to the right, beta: the MPO bond, b: psi's bond) starts as the right boundary (level 0); at
    site i = L-1 .. 1 the matrix
        X[(alpha, a), (s', k)] = sum_{s, b, beta} W_i[alpha, s', s, beta] psi_i[a, s, b] C[k, beta, b]
    is split by an FP64 SVD truncated like every bond of the fit (svd_truncate: k' = min(Dmax,
    #{sigma > cutoff sigma_1}) >= 1), the site becomes V^dag (k', s', k) and the carry (U S)^T
    (k', alpha, a). Site 0 is X at the left boundary level alpha = 0; it holds the norm.
    Returns (sites, stats) with stats = dict(discarded (per bond L-1 .. 1), bond_dims)."""
    L = len(psi)
    if not isinstance(Ws, (list, tuple)):
        Ws = [Ws] * L
    C = boundary_env(Ws[-1].shape[3])
    out = [None] * L
    discarded = []
    for i in range(L - 1, 0, -1):
        X = np.einsum('ypsz,asb,kzb->yapk', Ws[i], psi[i], C)
        y, a, p, k = X.shape
        U, S, Vh, disc = svd_truncate(X.reshape(y * a, p * k), Dmax, cutoff)
        discarded.append(disc)
        kk = S.size
        out[i] = Vh.reshape(kk, p, k)
        C = (U * S[None, :]).T.reshape(kk, y, a)
    X = np.einsum('ypsz,asb,kzb->yapk', Ws[0], psi[0], C)
    out[0] = X[0].reshape(psi[0].shape[0], X.shape[2], X.shape[3])
    dims = [1] + [out[i].shape[2] for i in range(L)]
    return out, dict(discarded=discarded, bond_dims=dims)


def fit_step(psi, Ws, Dmax: int, nsweeps: int = 2, cutoff: float = 1e-14, guess=None):
    """One time step: variational two-site fit of W|psi> at bonds <= Dmax (module docstring).

    psi: list of L site tensors; Ws: one MPO tensor or a list of L; guess: the starting phi, whose
    sites 1 .. L-1 must be right-orthonormal (default: psi right-canonicalised; zipup_guess gives
    another); returns (phi, stats) with phi normalised (unless W|psi> projects to zero) and
    stats = dict(norm, discarded (per visit), bond_dims)."""
    L = len(psi)
    if not isinstance(Ws, (list, tuple)):
        Ws = [Ws] * L
    if L == 1:
        phi0 = np.einsum('apsb,xsy->xpy', Ws[0][:1, :, :, :1], psi[0])  # boundary level 0 in and out
        n = np.linalg.norm(phi0)
        return [phi0 / n if n > 0 else phi0], dict(norm=float(n), discarded=[], bond_dims=[1, 1])
    phi = right_canonicalize(psi) if guess is None else [m.copy() for m in guess]
    Lenv = [None] * (L + 1)
    Renv = [None] * (L + 1)
    Lenv[0] = boundary_env(Ws[0].shape[0])
    Renv[L] = boundary_env(Ws[-1].shape[3])
    for i in range(L - 1, 1, -1):
        Renv[i] = env_right(Renv[i + 1], phi[i], Ws[i], psi[i])
    discarded = []
    S = None
    for _ in range(nsweeps):
        for i in range(0, L - 1):  # left to right
            th = theta_two_site(Lenv[i], psi[i], Ws[i], psi[i + 1], Ws[i + 1], Renv[i + 2])
            a, p, q, c = th.shape
            U, S, Vh, disc = svd_truncate(th.reshape(a * p, q * c), Dmax, cutoff)
            discarded.append(disc)
            k = S.size
            phi[i] = U.reshape(a, p, k)
            phi[i + 1] = (S[:, None] * Vh).reshape(k, q, c)
            if i < L - 2:
                Lenv[i + 1] = env_left(Lenv[i], phi[i], Ws[i], psi[i])
        for i in range(L - 2, -1, -1):  # right to left
            th = theta_two_site(Lenv[i], psi[i], Ws[i], psi[i + 1], Ws[i + 1], Renv[i + 2])
            a, p, q, c = th.shape
            U, S, Vh, disc = svd_truncate(th.reshape(a * p, q * c), Dmax, cutoff)
            discarded.append(disc)
            k = S.size
            phi[i] = (U * S[None, :]).reshape(a, p, k)
            phi[i + 1] = Vh.reshape(k, q, c)
            if i > 0:
                Renv[i + 1] = env_right(Renv[i + 2], phi[i + 1], Ws[i + 1], psi[i + 1])
    norm = float(np.linalg.norm(S))
    if norm > 0:
        phi[0] = phi[0] / norm
    dims = [1] + [phi[i].shape[2] for i in range(L)]
    return phi, dict(norm=norm, discarded=discarded, bond_dims=dims)


def overlap(bra, ket) -> complex:
    """<bra|ket> of two open-boundary MPS (transfer-matrix contraction)."""
    E = np.ones((1, 1), dtype=np.complex128)
    for A, B in zip(bra, ket):
        E = np.tensordot(E, A.conj(), axes=([0], [0]))        # [y, s, u]
        E = np.tensordot(E, B, axes=([0, 1], [0, 1]))         # [u, v]
    return complex(E[0, 0])


def norm(ms) -> float:
    return float(np.sqrt(abs(overlap(ms, ms))))


def expect_local(ms, op, site: int) -> complex:
    """<psi| op_site |psi> / <psi|psi>."""
    E = np.ones((1, 1), dtype=np.complex128)
    for j, A in enumerate(ms):
        B = np.tensordot(op, A, axes=([1], [1])).transpose(1, 0, 2) if j == site else A
        E = np.tensordot(E, A.conj(), axes=([0], [0]))
        E = np.tensordot(E, B, axes=([0, 1], [0, 1]))
    return complex(E[0, 0]) / overlap(ms, ms)


def mpo_expectation(ms, Wsites, left, right) -> complex:
    """<psi| O |psi> for an MPO O = l . W_1 ... W_L . r."""
    return mpo_overlap(ms, Wsites, ms, left, right)


def mpo_overlap(bra, Wsites, ket, left, right) -> complex:
    """<bra| O |ket> for an MPO O = l . W_1 ... W_L . r (left environments from the left end)."""
    E = np.einsum('a,xy->xay', left, np.ones((1, 1), dtype=np.complex128))
    for A, W, B in zip(bra, Wsites, ket):
        E = env_left(E, A, W, B)
    return complex(np.einsum('xay,a->', E, right))


def applied_norm2(psi, Ws) -> float:
    """||W psi||^2 = <psi| W^dag W |psi> through a double-layer environment
    E[bra, mpo (conjugated layer), mpo, ket]; boundary level 0 on both MPO layers."""
    L = len(psi)
    if not isinstance(Ws, (list, tuple)):
        Ws = [Ws] * L
    w = Ws[0].shape[0]
    E = np.zeros((1, w, w, 1), dtype=np.complex128)
    E[0, 0, 0, 0] = 1.0
    for A, W in zip(psi, Ws):
        T = np.tensordot(E, A, axes=([3], [0]))                    # [x, q, a, t, v]
        T = np.tensordot(T, W, axes=([2, 3], [0, 2]))              # [x, q, v, p, b]
        T = np.tensordot(T, W.conj(), axes=([1, 3], [0, 1]))       # [x, v, b, s, r]
        E = np.tensordot(A.conj(), T, axes=([0, 1], [0, 3]))       # [u, v, b, r]
        E = E.transpose(0, 3, 2, 1)
    return float(E[0, 0, 0, 0].real)


def local_one_site(Lenv, M, W, Renv):
    """Projected one-site tensor  M'[a', s', b'] = sum L[a', alpha, a] M[a, s, b] W[alpha, s', s, beta] R[b', beta, b]:
    the optimal site of the variational fit at fixed bonds, given the other sites (Sec. 2.2, Table 1
    "variational" row)."""
    return np.einsum('xay,ysb,apsg,ugb->xpu', Lenv, M, W, Renv, optimize=_EINSUM)


def fit_step_one_site(psi, Ws, nsweeps: int = 2, guess=None):
    """One time step by the one-site variational fit at the fixed bond dimensions of psi
    (Sec. 2.2; Sec. 8.2 keeps the bond dimension fixed). Readings (the paper leaves them open):
      * guess phi = psi brought to right-canonical form (as for the two-site fit);
      * a sweep is a left-to-right pass over the sites 0 .. L-2, where each site's optimal tensor
        (local_one_site) is replaced by the Q factor of its QR decomposition (rows (a', s'),
        columns b'; FP64), followed by a right-to-left pass over the sites L-1 .. 1, where it is
        replaced by the adjoint Q factor of the QR of its adjoint (rows a', columns (s', b'));
        the triangular factors are dropped (the next site is recomputed from the new environment);
      * after the last sweep the optimal tensor of site 0 completes phi; its norm is
        |<phi_hat|W psi>| and phi is normalised.
    Bonds must satisfy bond[i+1] <= d bond[i] after the guess (they do for the states a two-site
    fit produces). Returns (phi, stats) with stats = dict(norm, norms (of every local tensor, in
    visiting order), bond_dims). guess: another starting state (default psi) of the same length,
    whose bonds the result keeps."""
    L = len(psi)
    if not isinstance(Ws, (list, tuple)):
        Ws = [Ws] * L
    phi = right_canonicalize(psi if guess is None else guess)
    d = psi[0].shape[1]
    for i in range(L - 1):
        if phi[i].shape[2] > d * phi[i].shape[0]:
            raise ValueError("one-site fit: bond %d exceeds d times bond %d" % (i + 1, i))
    Lenv = [None] * (L + 1)
    Renv = [None] * (L + 1)
    Lenv[0] = boundary_env(Ws[0].shape[0])
    Renv[L] = boundary_env(Ws[-1].shape[3])
    for i in range(L - 1, 0, -1):
        Renv[i] = env_right(Renv[i + 1], phi[i], Ws[i], psi[i])
    norms = []
    for _ in range(nsweeps):
        for i in range(0, L - 1):  # left to right
            M = local_one_site(Lenv[i], psi[i], Ws[i], Renv[i + 1])
            norms.append(float(np.linalg.norm(M)))
            a, p, b = M.shape
            Q, _ = np.linalg.qr(M.reshape(a * p, b))
            phi[i] = Q.reshape(a, p, b)
            Lenv[i + 1] = env_left(Lenv[i], phi[i], Ws[i], psi[i])
        for i in range(L - 1, 0, -1):  # right to left
            M = local_one_site(Lenv[i], psi[i], Ws[i], Renv[i + 1])
            norms.append(float(np.linalg.norm(M)))
            a, p, b = M.shape
            Q, _ = np.linalg.qr(M.reshape(a, p * b).conj().T)
            phi[i] = Q.conj().T.reshape(a, p, b)
            Renv[i] = env_right(Renv[i + 1], phi[i], Ws[i], psi[i])
    M = local_one_site(Lenv[0], psi[0], Ws[0], Renv[1])
    norm = float(np.linalg.norm(M))
    norms.append(norm)
    phi[0] = M / norm if norm > 0 else M
    dims = [1] + [phi[i].shape[2] for i in range(L)]
    return phi, dict(norm=norm, norms=norms, bond_dims=dims)


def frozen_bonds(bond_dims, d: int, Dmax: int):
    """frozen[b] (b = 0 .. L): bond b is at its largest value min(Dmax, d^b, d^(L-b)) (the two ends
    always)."""
    L = len(bond_dims) - 1
    out = [True] * (L + 1)
    for b in range(1, L):
        out[b] = bond_dims[b] == min(Dmax, d ** min(b, L - b))
    return out


def fit_step_mixed(psi, Ws, Dmax: int, nsweeps: int = 2, cutoff: float = 1e-14):
    """One time step with the update chosen per position (our reading for states whose bonds are
    still growing; Sec. 2.2 gives both fits, Sec. 8.2 keeps the bond dimension fixed): the bonds
    at their largest value in the right-canonicalised guess are frozen; the sweeps visit the
    positions of the two-site fit (fit_step), and a position whose site has both bonds frozen --
    site i going left to right, site i + 1 going right to left -- takes the one-site update of
    that site (fit_step_one_site: QR of its projected tensor), every other position the two-site
    update (SVD truncation at Dmax, which may grow its bond). When the last visit is a one-site
    update, site 0's projected tensor completes phi as in the one-site fit. If a two-site update
    leaves a frozen bond below its starting value, the one-site updates next to it would no longer
    see the bond they were planned for: the step is then the plain two-site fit instead.
    With every bond frozen this is fit_step_one_site, with none fit_step. Returns (phi, stats)
    with stats = dict(norm, discarded (per visit, 0 for one-site visits), bond_dims, kinds (1 or 2
    per visit), fallback)."""
    L = len(psi)
    if not isinstance(Ws, (list, tuple)):
        Ws = [Ws] * L
    d = psi[0].shape[1]
    phi = right_canonicalize(psi)
    start = [1] + [phi[i].shape[2] for i in range(L)]
    fz = frozen_bonds(start, d, Dmax)
    if L == 1 or not any(fz[i] and fz[i + 1] for i in range(L)):
        ref, st = fit_step(psi, Ws, Dmax, nsweeps, cutoff)
        return ref, dict(st, kinds=[2] * len(st["discarded"]), fallback=False)
    Lenv = [None] * (L + 1)
    Renv = [None] * (L + 1)
    Lenv[0] = boundary_env(Ws[0].shape[0])
    Renv[L] = boundary_env(Ws[-1].shape[3])
    for i in range(L - 1, 0, -1):
        Renv[i] = env_right(Renv[i + 1], phi[i], Ws[i], psi[i])
    discarded, kinds = [], []
    S = None
    last_one = False

    def shrunk(b, k):  # a two-site update left the frozen bond b below its starting value
        return fz[b] and k < start[b]

    for _ in range(nsweeps):
        for i in range(0, L - 1):  # left to right
            if fz[i] and fz[i + 1]:
                M = local_one_site(Lenv[i], psi[i], Ws[i], Renv[i + 1])
                a, p, b = M.shape
                Q, _ = np.linalg.qr(M.reshape(a * p, b))
                phi[i] = Q.reshape(a, p, b)
                discarded.append(0.0)
                kinds.append(1)
            else:
                th = theta_two_site(Lenv[i], psi[i], Ws[i], psi[i + 1], Ws[i + 1], Renv[i + 2])
                a, p, q, c = th.shape
                U, S, Vh, disc = svd_truncate(th.reshape(a * p, q * c), Dmax, cutoff)
                k = S.size
                if shrunk(i + 1, k):
                    ref, st = fit_step(psi, Ws, Dmax, nsweeps, cutoff)
                    return ref, dict(st, kinds=[2] * len(st["discarded"]), fallback=True)
                discarded.append(disc)
                kinds.append(2)
                phi[i] = U.reshape(a, p, k)
                phi[i + 1] = (S[:, None] * Vh).reshape(k, q, c)
            Lenv[i + 1] = env_left(Lenv[i], phi[i], Ws[i], psi[i])
        for i in range(L - 2, -1, -1):  # right to left
            if fz[i + 1] and fz[i + 2]:
                M = local_one_site(Lenv[i + 1], psi[i + 1], Ws[i + 1], Renv[i + 2])
                a, p, b = M.shape
                Q, _ = np.linalg.qr(M.reshape(a, p * b).conj().T)
                phi[i + 1] = Q.conj().T.reshape(a, p, b)
                discarded.append(0.0)
                kinds.append(1)
                last_one = True
            else:
                th = theta_two_site(Lenv[i], psi[i], Ws[i], psi[i + 1], Ws[i + 1], Renv[i + 2])
                a, p, q, c = th.shape
                U, S, Vh, disc = svd_truncate(th.reshape(a * p, q * c), Dmax, cutoff)
                k = S.size
                if shrunk(i + 1, k):
                    ref, st = fit_step(psi, Ws, Dmax, nsweeps, cutoff)
                    return ref, dict(st, kinds=[2] * len(st["discarded"]), fallback=True)
                discarded.append(disc)
                kinds.append(2)
                phi[i] = (U * S[None, :]).reshape(a, p, k)
                phi[i + 1] = Vh.reshape(k, q, c)
                last_one = False
            Renv[i + 1] = env_right(Renv[i + 2], phi[i + 1], Ws[i + 1], psi[i + 1])
    if last_one:  # site 0's projected tensor completes phi (one-site fit)
        M = local_one_site(Lenv[0], psi[0], Ws[0], Renv[1])
        norm = float(np.linalg.norm(M))
        phi[0] = M / norm if norm > 0 else M
    else:
        norm = float(np.linalg.norm(S))
        if norm > 0:
            phi[0] = phi[0] / norm
    dims = [1] + [phi[i].shape[2] for i in range(L)]
    return phi, dict(norm=norm, discarded=discarded, bond_dims=dims, kinds=kinds, fallback=False)
