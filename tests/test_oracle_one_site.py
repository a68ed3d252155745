"""Pins of the oracle's one-site variational fit at fixed bonds (Sec. 2.2; Sec. 8.2 keeps the bond
dimension fixed), against facts that do not come from its own formulas:
  * brute force: with complete bonds (bond i = min(d^i, d^(L-i))) one sweep reproduces the dense
    W|psi> / ||W psi|| exactly, and the fitted norm is ||W psi||;
  * alternating maximisation: the norm of each local optimum, |<phi_hat|W psi>| with the other
    sites fixed, never decreases along the sweeps;
  * started from the two-site fit's result (same bonds), the one-site fit never does worse than it;
  * tau = 0 (W = identity): the fit returns psi itself.
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


@pytest.mark.parametrize("L,chi,N", [(6, 1, 2), (7, 2, 3), (5, 2, 1)])
def test_complete_bonds_reproduce_dense(L, chi, N):
    rng = np.random.default_rng(60 + L + chi)
    H = wl.random_blocks(rng, 2, chi)
    W = ompo.build_mpo(H, N, 0.07 - 0.05j, "V2")
    psi = _normalise(wl.random_mps(rng, L, 2, 2 ** L))  # complete bonds
    v = dense.dense_evolution_mpo(W, L) @ dense.mps_to_dense(psi)
    phi, st = ofit.fit_step_one_site(psi, W, nsweeps=1)
    f = dense.mps_to_dense(phi)
    assert abs(st["norm"] - np.linalg.norm(v)) < 1e-12 * np.linalg.norm(v)
    assert 1 - abs(np.vdot(f, v)) ** 2 / np.linalg.norm(v) ** 2 < 1e-12


@pytest.mark.parametrize("seed", [1, 2])
def test_local_optima_never_decrease(seed):
    rng = np.random.default_rng(seed)
    L, D = 10, 6
    H = wl.random_hermitian_blocks(rng, 2, 2)
    W = ompo.build_mpo(H, 2, -0.2j, "V2")
    psi = _normalise(wl.random_mps(rng, L, 2, D))
    _, st = ofit.fit_step_one_site(psi, W, nsweeps=3)
    n = np.array(st["norms"])
    assert np.all(np.diff(n) >= -1e-12 * n[:-1]), np.diff(n).min()
    assert n[-1] > n[0]  # truncated bonds: the sweeps do improve on the guess


def test_not_worse_than_two_site_start():
    rng = np.random.default_rng(9)
    L, D = 10, 8
    H = wl.tfim(1.3)
    W = ompo.build_mpo(H, 2, -0.3j, "V2")
    psi = _normalise(wl.random_mps(rng, L, 2, D))
    two, st2 = ofit.fit_step(psi, W, Dmax=D)
    one, st1 = ofit.fit_step_one_site(psi, W, nsweeps=2, guess=two)
    assert [m.shape for m in one] == [m.shape for m in two]
    assert st1["norm"] >= st2["norm"] * (1 - 1e-12)
    v = dense.dense_evolution_mpo(W, L) @ dense.mps_to_dense(psi)
    fid = lambda ms: abs(np.vdot(dense.mps_to_dense(ms), v)) ** 2 / np.linalg.norm(v) ** 2  # noqa: E731
    assert fid(one) >= fid(two) - 1e-12


def test_identity_returns_input():
    rng = np.random.default_rng(4)
    L, D = 8, 5
    psi = _normalise(wl.random_mps(rng, L, 2, D))
    W = ompo.build_mpo(wl.tfim(1.0), 2, 0.0, "V2")
    phi, st = ofit.fit_step_one_site(psi, W)
    assert abs(st["norm"] - 1) < 1e-12
    assert 1 - abs(ofit.overlap(phi, psi)) ** 2 < 1e-12
