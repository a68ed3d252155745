"""Pins of the oracle's fit with the update chosen per position (fit_step_mixed: one-site updates
at sites whose bonds are both at their largest value, two-site updates elsewhere), against facts
that do not come from its own formulas:
  * its two limits: with every bond frozen it is the one-site fit, with none the two-site fit
    (each pinned on its own);
  * brute force: with Dmax at the complete bond dimension, a state with one bond below it is fitted
    exactly (one-site visits on the complete bonds, two-site visits growing the other), against the
    dense W|psi>;
  * with truncation, the mixed fit's overlap with W|psi> is at least that of its guess, and its
    statistics name the updates it took;
  * a frozen bond that a two-site update leaves below its starting value makes the step the plain
    two-site fit.
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


def _same(a, b, tol=1e-12):
    return all(x.shape == y.shape and np.max(np.abs(x - y)) <= tol * max(1.0, np.max(np.abs(y))) for x, y in zip(a, b))


def test_frozen_bonds():
    assert ofit.frozen_bonds([1, 2, 4, 5, 4, 2, 1], 2, 8) == [True, True, True, False, True, True, True]
    assert ofit.frozen_bonds([1, 2, 4, 6, 6, 4, 2, 1], 2, 6) == [True] * 8
    assert ofit.frozen_bonds([1, 2, 3, 3, 2, 1], 2, 4) == [True, True, False, False, True, True]


def test_all_frozen_is_the_one_site_fit():
    rng = np.random.default_rng(11)
    L, D = 9, 8
    psi = _normalise(wl.random_mps(rng, L, 2, D))  # every bond at min(D, 2^b, 2^(L-b))
    W = ompo.build_mpo(wl.random_blocks(rng, 2, 2), 2, 0.05 - 0.08j, "V2")
    a, sa = ofit.fit_step_mixed(psi, W, D)
    b, sb = ofit.fit_step_one_site(psi, W)
    assert set(sa["kinds"]) == {1} and not sa["fallback"]
    assert _same(a, b) and abs(sa["norm"] - sb["norm"]) < 1e-13 * sb["norm"]


def test_none_frozen_is_the_two_site_fit():
    rng = np.random.default_rng(12)
    L, D = 8, 8
    dims = [1, 1, 2, 3, 3, 3, 2, 1, 1]  # every inner bond below its largest value
    psi = _normalise(wl.random_mps(rng, L, 2, D, dims))
    W = ompo.build_mpo(wl.random_blocks(rng, 2, 1), 2, -0.1j, "V2")
    a, sa = ofit.fit_step_mixed(psi, W, D)
    b, sb = ofit.fit_step(psi, W, D)
    assert set(sa["kinds"]) == {2}
    assert _same(a, b) and abs(sa["norm"] - sb["norm"]) < 1e-13 * sb["norm"]


@pytest.mark.parametrize("L,dims,N", [(6, [1, 2, 4, 5, 4, 2, 1], 2), (7, [1, 2, 3, 8, 8, 4, 2, 1], 3),
                                      (8, [1, 2, 4, 8, 9, 8, 4, 2, 1], 1)])
def test_complete_dmax_is_exact(L, dims, N):
    rng = np.random.default_rng(70 + L)
    D = 2 ** (L // 2)
    psi = _normalise(wl.random_mps(rng, L, 2, D, dims))
    W = ompo.build_mpo(wl.random_blocks(rng, 2, 2), N, 0.06 - 0.04j, "V2")
    v = dense.dense_evolution_mpo(W, L) @ dense.mps_to_dense(psi)
    phi, st = ofit.fit_step_mixed(psi, W, D)
    assert 1 in st["kinds"] and 2 in st["kinds"] and not st["fallback"]
    f = dense.mps_to_dense(phi)
    assert abs(st["norm"] - np.linalg.norm(v)) < 1e-12 * np.linalg.norm(v)
    assert 1 - abs(np.vdot(f, v)) ** 2 / np.linalg.norm(v) ** 2 < 1e-12
    assert abs(np.linalg.norm(f) - 1) < 1e-12


def test_truncating_step_improves_on_its_guess():
    rng = np.random.default_rng(5)
    L, D = 12, 6
    caps = [min(D, 2 ** min(b, L - b)) for b in range(L + 1)]
    dims = list(caps)
    dims[5], dims[6] = 4, 5  # two bonds still growing, the rest at their largest value
    psi = _normalise(wl.random_mps(rng, L, 2, D, dims))
    W = ompo.build_mpo(wl.random_blocks(rng, 2, 2), 2, -0.15j, "V2")
    phi, st = ofit.fit_step_mixed(psi, W, D)
    kinds = st["kinds"]
    assert len(kinds) == 4 * (L - 1) and kinds.count(1) > kinds.count(2) > 0
    # the visit pattern: one-site exactly where the site has both bonds frozen (bonds 5 and 6
    # growing: sites 4, 5 and 6 touch one of them and take two-site updates, going either way)
    lr = [2 if i in (4, 5, 6) else 1 for i in range(L - 1)]              # position i: site i
    rl = [2 if i + 1 in (4, 5, 6) else 1 for i in range(L - 2, -1, -1)]  # position i: site i + 1
    assert kinds == (lr + rl) * 2, kinds
    assert all(d == 0.0 for d, k in zip(st["discarded"], kinds) if k == 1)
    # the fitted overlap beats the guess's: |<phi|W psi>| >= |<psi_hat|W psi>|
    e0 = np.zeros(W.shape[0], dtype=np.complex128)
    e0[0] = 1.0  # boundary level 0 in and out
    wpsi_on = lambda bra: abs(ofit.mpo_overlap(bra, [W] * L, psi, e0, e0)) / np.sqrt(ofit.overlap(bra, bra).real)
    assert st["norm"] >= wpsi_on(psi) * (1 - 1e-12)
    assert abs(wpsi_on(phi) - st["norm"]) < 1e-10 * st["norm"]
    assert max(st["bond_dims"]) <= D


def test_shrinking_frozen_bond_falls_back_to_two_site():
    # psi is a product state padded to bond 2 everywhere near the left end: bond 1 is at its
    # largest value (2) but its Schmidt rank is 1, which the two-site update of that bond finds
    rng = np.random.default_rng(9)
    L, D = 6, 4
    dims = [1, 2, 3, 4, 4, 2, 1]
    psi = wl.random_mps(rng, L, 2, D, dims)
    psi[0] = np.zeros_like(psi[0])
    psi[0][0, :, 0] = [0.6, 0.8]  # site 0 couples only to index 0 of bond 1
    psi = _normalise(psi)
    W = ompo.build_mpo(wl.random_blocks(rng, 2, 1), 1, 0.0, "V2")  # tau = 0: W is the identity
    assert ofit.frozen_bonds([1] + [m.shape[2] for m in ofit.right_canonicalize(psi)], 2, D)[1]
    phi, st = ofit.fit_step_mixed(psi, W, D)
    ref, _ = ofit.fit_step(psi, W, D)
    assert st["fallback"] and _same(phi, ref)
