"""Pins of the oracle's zip-up guess (Sec. 2.2, Table 1 zip-up row), against facts that do not
come from its own formulas:
  * brute force: without truncation the zip-up state is the dense W|psi> (the MPO applied as a
    dense operator), for first- to third-order MPOs with chi = 1, 2;
  * its sites 1 .. L-1 are right-orthonormal;
  * W = identity on a left-canonical psi: each SVD of the zip is the Schmidt decomposition of the
    current state across that bond, so the zip-up equals the dense sequential truncation from the
    right end (Eckart-Young at every cut), with the discarded weights of those SVDs;
  * used as the guess of the two-site fit at complete bonds, the fit reproduces W|psi> exactly.
"""
import numpy as np
import pytest

from oracle import dense, fit as ofit, mpo as ompo
from paper_2302_14181_amd import workloads as wl


def _normalise(ms):
    n = ofit.norm(ms)
    out = [m.copy() for m in ms]
    out[0] = out[0] / n
    return out


@pytest.mark.parametrize("L,chi,N", [(6, 1, 2), (5, 2, 3), (6, 2, 1), (4, 1, 3)])
def test_untruncated_zipup_is_dense_w_psi(L, chi, N):
    rng = np.random.default_rng(80 + L + 3 * chi + N)
    H = wl.random_blocks(rng, 2, chi)
    W = ompo.build_mpo(H, N, 0.09 - 0.06j, "V2")
    psi = _normalise(wl.random_mps(rng, L, 2, 3))
    v = dense.dense_evolution_mpo(W, L) @ dense.mps_to_dense(psi)
    z, st = ofit.zipup_guess(psi, W, Dmax=10 ** 6, cutoff=0.0)
    assert np.max(np.abs(dense.mps_to_dense(z) - v)) < 1e-12 * np.max(np.abs(v))
    assert max(st["discarded"]) < 1e-26
    for i in range(1, L):
        M = z[i].reshape(z[i].shape[0], -1)
        assert np.allclose(M @ M.conj().T, np.eye(M.shape[0]), atol=1e-12), i


def _left_canonical(rng, L, d, D):
    ms = wl.random_mps(rng, L, d, D)
    out = []
    carry = np.ones((1, 1), dtype=np.complex128)
    for i, M in enumerate(ms):
        M = np.einsum('xa,asb->xsb', carry, M)
        a, s, b = M.shape
        if i == L - 1:
            out.append(M / np.linalg.norm(M))
            break
        Q, R = np.linalg.qr(M.reshape(a * s, b))
        out.append(Q.reshape(a, s, Q.shape[1]))
        carry = R
    return out


def test_identity_zipup_is_sequential_schmidt_truncation():
    rng = np.random.default_rng(7)
    L, d, D, Dmax = 7, 2, 8, 3
    psi = _left_canonical(rng, L, d, D)
    ident = np.eye(d, dtype=np.complex128).reshape(1, d, d, 1)
    z, st = ofit.zipup_guess(psi, ident, Dmax=Dmax, cutoff=0.0)
    v = dense.mps_to_dense(psi)
    disc = []
    for cut in range(L - 1, 0, -1):  # bond between sites cut-1 and cut, from the right end
        M = v.reshape(d ** cut, d ** (L - cut))
        U, S, Vh = np.linalg.svd(M, full_matrices=False)
        k = min(Dmax, S.size)
        disc.append(float(np.sum(S[k:] ** 2) / np.sum(S ** 2)))
        v = ((U[:, :k] * S[:k]) @ Vh[:k]).reshape(-1)
    f = dense.mps_to_dense(z)
    assert np.max(np.abs(f - v)) < 1e-12
    assert np.allclose(st["discarded"], disc, rtol=1e-9, atol=1e-15)
    assert max(st["discarded"]) > 1e-3  # the case truncates
    assert st["bond_dims"] == [1, 2, 3, 3, 3, 3, 2, 1]


@pytest.mark.parametrize("L,N", [(6, 2), (5, 3)])
def test_fit_from_zipup_guess_complete_bonds(L, N):
    rng = np.random.default_rng(90 + L)
    W = ompo.build_mpo(wl.tfim(1.3), N, -0.2j, "V2")
    psi = _normalise(wl.random_mps(rng, L, 2, 2))
    v = dense.dense_evolution_mpo(W, L) @ dense.mps_to_dense(psi)
    z, _ = ofit.zipup_guess(psi, W, Dmax=2 ** L, cutoff=0.0)
    phi, st = ofit.fit_step(psi, W, Dmax=2 ** L, nsweeps=1, guess=z)
    f = dense.mps_to_dense(phi)
    assert abs(st["norm"] - np.linalg.norm(v)) < 1e-12 * np.linalg.norm(v)
    assert 1 - abs(np.vdot(f, v)) ** 2 / np.linalg.norm(v) ** 2 < 1e-13
