"""Pins of the block-sparse U(1) oracle (dictionaries of blocks, oracle/u1.py) against the dense
oracle and against brute force, on the XXZ chain (Sec. 2.4) with seeded random U(1) states:
  * the block-sparse fit equals the dense fit of the same dense state (gauge-invariant overlap,
    fitted norm, discarded weights), with and without truncation;
  * without truncation it reproduces the dense W|psi> / ||W psi|| (brute force);
  * charge: every block of the result obeys q(b) = q(a) + q(s), and the dense vector of the result
    has no weight outside the input's charge sector.
"""
import numpy as np
import pytest

from oracle import dense, fit as ofit, mpo as ompo, u1
from paper_2302_14181_amd import workloads as wl


def _case(L, n_up, D0, seed, order=2, tau=-0.1j):
    H = wl.xxz(0.5)
    qp = H.phys_charge
    W = ompo.build_mpo(H, order, tau, "V2")
    lc = ompo.level_charges(H, order, tau, "V2")
    tables = wl.u1_sector_tables(L, n_up, D0, nsec=7, seed=seed)
    psi = wl.random_u1_mps(np.random.default_rng(seed), tables, qp)
    return H, qp, W, lc, tables, psi


@pytest.mark.parametrize("L,n_up,D0,Dmax", [(8, 4, 16, 6), (10, 5, 12, 8), (12, 6, 24, 16)])
def test_block_fit_equals_dense_fit(L, n_up, D0, Dmax):
    H, qp, W, lc, tables, psi = _case(L, n_up, D0, seed=L)
    phi_b, pb, sb = u1.fit_step(psi, tables, W, lc, qp, Dmax)
    for i in range(L):
        u1.check_blocks(phi_b[i], pb[i], pb[i + 1], qp)
    phi_d, sd = ofit.fit_step(u1.to_dense(psi, tables, qp), W, Dmax)
    a = u1.to_dense(phi_b, pb, qp)
    assert 1 - abs(ofit.overlap(a, phi_d)) ** 2 < 1e-12
    assert abs(sb["norm"] - sd["norm"]) < 1e-12 * sd["norm"]
    assert np.allclose(sb["discarded"], sd["discarded"], atol=1e-13)
    assert max(sd["discarded"]) > 1e-8  # the case does truncate
    assert all(sum(b.values()) <= Dmax for b in pb)


def test_untruncated_block_fit_is_dense_W_psi():
    L, n_up = 8, 4
    H, qp, W, lc, tables, psi = _case(L, n_up, 16, seed=3)
    v = dense.dense_evolution_mpo(W, L) @ dense.mps_to_dense(u1.to_dense(psi, tables, qp))
    phi, pb, st = u1.fit_step(psi, tables, W, lc, qp, Dmax=64)
    f = dense.mps_to_dense(u1.to_dense(phi, pb, qp))
    assert abs(st["norm"] - np.linalg.norm(v)) < 1e-12 * np.linalg.norm(v)
    assert 1 - abs(np.vdot(f, v)) ** 2 / np.linalg.norm(v) ** 2 < 1e-12
    # the charge sector: every basis state with weight has n_up up spins (up = index 0)
    nup = np.array([sum(1 for k in range(L) if not (i >> (L - 1 - k)) & 1) for i in range(2 ** L)])
    assert np.abs(f[nup != n_up]).max() < 1e-14
    assert abs(np.linalg.norm(f[nup == n_up]) - 1) < 1e-12
