"""Oracle: dense references for tiny chains (complex128).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def contract_mpo(W_sites, left: np.ndarray, right: np.ndarray) -> np.ndarray:
    """Dense operator  l . W_1 W_2 ... W_L . r  of a finite MPO (Sec. 2.1); site 1 is the most
    significant factor of the tensor-product basis. W_sites: list of (w_l, d, d, w_r) tensors."""
    X = np.einsum('a,apqb->pqb', left, W_sites[0])
    for W in W_sites[1:]:
        P, Q, _ = X.shape
        d = W.shape[1]
        X = np.einsum('pqb,bstc->psqtc', X, W).reshape(P * d, Q * d, W.shape[3])
    return np.einsum('pqb,b->pq', X, right)


def boundary(w: int, index: int = 0) -> np.ndarray:
    e = np.zeros(w, dtype=np.complex128)
    e[index] = 1.0
    return e


def dense_evolution_mpo(W: np.ndarray, L: int) -> np.ndarray:
    """Dense operator of the uniform time-evolution MPO on L sites, boundaries l = r = e_0 (Sec. 3)."""
    w = W.shape[0]
    return contract_mpo([W] * L, boundary(w), boundary(w))


def dense_hamiltonian(Hmpo: np.ndarray, L: int) -> np.ndarray:
    """Dense Hamiltonian from its level-(1,2,3) MPO: enter at level 1, leave at level 3."""
    w = Hmpo.shape[0]
    return contract_mpo([Hmpo] * L, boundary(w, 0), boundary(w, w - 1))


def local_op(op: np.ndarray, site: int, L: int) -> np.ndarray:
    d = op.shape[0]
    return np.kron(np.kron(np.eye(d ** site), op), np.eye(d ** (L - site - 1)))


def expm(tau: complex, H: np.ndarray) -> np.ndarray:
    """exp(tau H) for a dense matrix (scipy's Pade scaling-and-squaring)."""
    return scipy.linalg.expm(tau * H)


def expm_hermitian(tau: complex, H: np.ndarray) -> np.ndarray:
    """exp(tau H) for Hermitian H through its eigendecomposition."""
    lam, V = np.linalg.eigh(H)
    return (V * np.exp(tau * lam)) @ V.conj().T


def mps_to_dense(ms) -> np.ndarray:
    """State vector of an open-boundary MPS (left and right bonds of dimension 1)."""
    X = ms[0]
    for M in ms[1:]:
        a, p, b = X.shape
        X = np.einsum('apb,bsc->apsc', X, M).reshape(a, p * M.shape[1], M.shape[2])
    return X.reshape(-1)
