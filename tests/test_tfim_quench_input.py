"""The initial state of the L = 64 transverse-field Ising quench (tests/golden/tfim_g05_L64_ground.npz,
written by tests/golden/make_tfim_ground.py through the oracle alone), pinned to the exact
free-fermion ground energy of the open chain.

The open chain H = -sum_{i<L} Z_i Z_{i+1} - g sum_i X_i maps (Jordan-Wigner, after exchanging X and Z)
to the quadratic form sum c^dag A c + 1/2 sum (c^dag B c^dag + h.c.) - g L with A = tridiag(-1, 2g,
-1) and B antisymmetric (-1 above, +1 below the diagonal); its ground energy is -1/2 sum_k Lambda_k
with Lambda_k^2 the eigenvalues of (A - B)(A + B) (Lieb, Schultz and Mattis). The formula itself is
checked against dense diagonalisation first.
"""
import os

import numpy as np
import pytest

from oracle import dense, fit, mpo
from paper_2302_14181_amd import workloads as wl

FIXTURE = os.path.join(os.path.dirname(__file__), "golden", "tfim_g05_L64_ground.npz")


def free_fermion_ground_energy(L, g):
    A = np.diag(np.full(L, 2.0 * g)) - np.diag(np.ones(L - 1), 1) - np.diag(np.ones(L - 1), -1)
    B = -np.diag(np.ones(L - 1), 1) + np.diag(np.ones(L - 1), -1)
    M = (A - B) @ (A + B)
    lam = np.sqrt(np.clip(np.linalg.eigvalsh((M + M.T) / 2), 0.0, None))
    return -0.5 * float(lam.sum())


def load_fixture():
    z = np.load(FIXTURE)
    sites = [z[f"site_{i:03d}"] for i in range(64)]
    return sites, z


def mpo_energy(ms, H):
    Wh = mpo.hamiltonian_mpo(H)
    w = Wh.shape[0]
    left, right = np.zeros(w, complex), np.zeros(w, complex)
    left[0], right[w - 1] = 1.0, 1.0
    return float((fit.mpo_expectation(ms, [Wh] * len(ms), left, right) / fit.overlap(ms, ms)).real)


@pytest.mark.parametrize("L,g", [(6, 0.5), (8, 0.5), (8, 1.5)])
def test_free_fermion_formula_matches_dense_diagonalisation(L, g):
    Hd = dense.dense_hamiltonian(mpo.hamiltonian_mpo(wl.tfim(g)), L)
    assert abs(np.linalg.eigvalsh(Hd)[0] - free_fermion_ground_energy(L, g)) < 1e-12 * L


def test_quench_initial_state_is_the_g05_ground_state():
    sites, z = load_fixture()
    assert float(z["g"]) == 0.5 and float(z["tau"]) == -0.05
    assert all(s.shape[0] <= 128 and s.shape[2] <= 128 for s in sites)
    assert sites[0].shape[0] == 1 and sites[-1].shape[2] == 1
    assert abs(fit.norm(sites) - 1.0) < 1e-12
    e = mpo_energy(sites, wl.tfim(0.5))
    assert abs(e - float(z["energy"])) < 1e-10
    e0 = free_fermion_ground_energy(64, 0.5)
    # variational (not below the exact energy) and within the imaginary-time bias of an
    # order-2 step at tau = 0.05
    assert -1e-9 <= e - e0 < 1e-5
    # a ferromagnet at g = 0.5: <Z> well away from zero in the bulk
    assert fit.expect_local(sites, wl.SZ, 31).real > 0.9
