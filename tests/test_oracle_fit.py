"""Pins of the oracle's variational fit (one time step) by brute force on tiny chains and by
exact diagonalisation (the tiny transverse-field Ising configuration: L = 10, g = 1, order 2,
tau = 0.05, all-up start, D <= 16, 20 steps, two sweeps per step)."""
import numpy as np
import pytest

from oracle import dense, fit, mpo
from paper_2302_14181_amd import workloads as wl


def _normalise(ms):
    n = fit.norm(ms)
    out = [m.copy() for m in ms]
    out[0] = out[0] / n
    return out


def test_environment_contractions_against_dense():
    """<phi| W |psi> through left environments equals the dense overlap (random tensors)."""
    rng = np.random.default_rng(1)
    L = 5
    psi = wl.random_mps(rng, L, 2, 3)
    phi = wl.random_mps(rng, L, 2, 4)
    W = mpo.build_mpo(wl.random_blocks(rng, 2, 2), 2, 0.2 - 0.1j, "V2")
    Wd = dense.dense_evolution_mpo(W, L)
    ref = np.vdot(dense.mps_to_dense(phi), Wd @ dense.mps_to_dense(psi))
    E = fit.boundary_env(W.shape[0])
    for i in range(L):
        E = fit.env_left(E, phi[i], W, psi[i])
    assert abs(E[0, 0, 0] - ref) < 1e-12 * abs(ref)
    R = fit.boundary_env(W.shape[0])
    for i in range(L - 1, -1, -1):
        R = fit.env_right(R, phi[i], W, psi[i])
    assert abs(R[0, 0, 0] - ref) < 1e-12 * abs(ref)
    # the projected two-site tensor contracted with the bra sites gives the same number
    Lenv = fit.boundary_env(W.shape[0])
    Lenv = fit.env_left(Lenv, phi[0], W, psi[0])
    Renv = fit.boundary_env(W.shape[0])
    for i in range(L - 1, 2, -1):
        Renv = fit.env_right(Renv, phi[i], W, psi[i])
    th = fit.theta_two_site(Lenv, psi[1], W, psi[2], W, Renv)
    val = np.einsum('xpqu,xpy,yqu->', th, phi[1].conj(), phi[2].conj())
    assert abs(val - ref) < 1e-12 * abs(ref)


def test_right_canonical_form():
    rng = np.random.default_rng(2)
    psi = wl.random_mps(rng, 6, 2, 5)
    rc = fit.right_canonicalize(psi)
    for i in range(1, 6):
        a, d, b = rc[i].shape
        m = rc[i].reshape(a, d * b)
        assert np.allclose(m @ m.conj().T, np.eye(a), atol=1e-13)
    s1, s2 = dense.mps_to_dense(psi), dense.mps_to_dense(rc)
    assert np.max(np.abs(s1 - s2)) < 1e-13 * np.max(np.abs(s1))


@pytest.mark.parametrize("seed", [0, 1])
def test_fit_without_truncation_is_exact(seed):
    """With Dmax above every bond of W|psi>, two sweeps reproduce the dense W|psi>:
    infidelity <= 1e-12 and the pre-normalisation norm equals ||W psi|| (psi normalised)."""
    rng = np.random.default_rng(seed)
    L = 7
    psi = _normalise(wl.random_mps(rng, L, 2, 2))
    W = mpo.build_mpo(wl.random_blocks(rng, 2, 1), 2, 0.15 + 0.05j, "V2")
    target = dense.dense_evolution_mpo(W, L) @ dense.mps_to_dense(psi)
    phi, st = fit.fit_step(psi, W, Dmax=64, nsweeps=2)
    v = dense.mps_to_dense(phi)
    infid = 1 - abs(np.vdot(v, target)) ** 2 / (np.vdot(v, v).real * np.vdot(target, target).real)
    assert infid < 1e-12
    assert abs(st["norm"] - np.linalg.norm(target)) < 1e-12 * np.linalg.norm(target)
    assert abs(fit.norm(phi) - 1) < 1e-13
    assert max(st["discarded"]) < 1e-24
    assert abs(fit.applied_norm2(psi, W) - np.linalg.norm(target) ** 2) < 1e-12 * np.linalg.norm(target) ** 2


def test_truncated_fit_is_optimal_two_site():
    """With truncation, the fitted state is never worse than the guess and keeps <= Dmax."""
    rng = np.random.default_rng(3)
    L = 8
    psi = _normalise(wl.random_mps(rng, L, 2, 4))
    W = mpo.build_mpo(wl.random_blocks(rng, 2, 1), 2, 0.2, "V2")
    target = dense.dense_evolution_mpo(W, L) @ dense.mps_to_dense(psi)
    target /= np.linalg.norm(target)
    phi, st = fit.fit_step(psi, W, Dmax=4, nsweeps=2)
    assert max(st["bond_dims"]) <= 4
    fid = abs(np.vdot(dense.mps_to_dense(phi), target)) ** 2
    fid_guess = abs(np.vdot(dense.mps_to_dense(psi), target)) ** 2
    assert fid > fid_guess
    assert fid > 1 - 10 * max(st["discarded"]) * len(st["discarded"])
    # the reported norm is the overlap |<phi|W psi>| (phi normalised)
    tgt_unnorm = dense.dense_evolution_mpo(W, L) @ dense.mps_to_dense(psi)
    assert abs(abs(np.vdot(dense.mps_to_dense(phi), tgt_unnorm)) - st["norm"]) < 1e-12


def test_norm_conservation_order():
    """Unitary target (tau = -i dt): | ||W psi||^2 - 1 | = O(dt^(N+1)) per step."""
    H = wl.tfim(1.0)
    rng = np.random.default_rng(4)
    L = 8
    psi = _normalise(wl.random_mps(rng, L, 2, 4))
    for N in (1, 2, 3):
        dts = [0.1, 0.05]
        errs = [abs(fit.applied_norm2(psi, mpo.build_mpo(H, N, -1j * dt, "V2")) - 1) for dt in dts]
        slope = np.log(errs[0] / errs[1]) / np.log(2)
        assert slope > N + 1 - 0.2, (N, errs, slope)


def _tfim_config1(D, steps=20, dt=0.05):
    L = 10
    H = wl.tfim(1.0)
    W = mpo.build_mpo(H, 2, -1j * dt, "V2")
    psi = wl.all_up(L)
    states = [psi]
    for _ in range(steps):
        psi, st = fit.fit_step(psi, W, Dmax=D, nsweeps=2)
        states.append(psi)
    return H, W, states


@pytest.mark.slow
def test_config1_against_stepwise_dense_and_exact():
    """Tiny TFIM configuration: (i) with D = 32 (no truncation on L = 10) the MPS equals the
    stepwise dense W^k psi0 (normalised) to 1e-10 in infidelity; with D = 16 the gap is only
    truncation; (ii) the dense W^k psi0 follows exp(-i t H) psi0 with a global error that
    falls like dt^2 for the second-order operator."""
    L = 10
    H, W, states32 = _tfim_config1(32)
    Wd = dense.dense_evolution_mpo(W, L)
    v = dense.mps_to_dense(wl.all_up(L))
    for k in range(1, 21):
        v = Wd @ v
        v /= np.linalg.norm(v)
        s = dense.mps_to_dense(states32[k])
        assert 1 - abs(np.vdot(s, v)) ** 2 < 1e-10
    _, _, states16 = _tfim_config1(16)
    s16 = dense.mps_to_dense(states16[-1])
    assert 1 - abs(np.vdot(s16, v)) ** 2 < 1e-6
    # exact evolution and the global error order of the dense stepper
    Hd = dense.dense_hamiltonian(mpo.hamiltonian_mpo(H), L)
    v0 = dense.mps_to_dense(wl.all_up(L))
    errs = []
    for dt in (0.1, 0.05, 0.025):
        Wd_dt = dense.dense_evolution_mpo(mpo.build_mpo(H, 2, -1j * dt, "V2"), L)
        x = v0.copy()
        for _ in range(int(round(1.0 / dt))):
            x = Wd_dt @ x
        exact = dense.expm_hermitian(-1j * 1.0, Hd) @ v0
        errs.append(np.linalg.norm(x - exact))
    slopes = [np.log(errs[i] / errs[i + 1]) / np.log(2) for i in range(2)]
    assert min(slopes) > 2 - 0.2, (errs, slopes)
    # energy is conserved up to the order of the scheme
    E0 = np.vdot(v0, Hd @ v0).real
    sT = dense.mps_to_dense(states32[-1])
    assert abs(np.vdot(sT, Hd @ sT).real - E0) < 5e-3


def test_fit_observables_gauge_invariant():
    """<Z_j> computed from the MPS matches the dense state."""
    rng = np.random.default_rng(6)
    psi = _normalise(wl.random_mps(rng, 6, 2, 3))
    v = dense.mps_to_dense(psi)
    for j in (0, 3, 5):
        ref = np.vdot(v, dense.local_op(wl.SZ, j, 6) @ v).real
        assert abs(fit.expect_local(psi, wl.SZ, j).real - ref) < 1e-13


def test_mpo_overlap_equals_dense():
    """<bra| O |ket> through the environments equals the dense bra^dag O ket (different bonds)."""
    rng = np.random.default_rng(12)
    L = 6
    bra, ket = wl.random_mps(rng, L, 2, 3), wl.random_mps(rng, L, 2, 5)
    W = mpo.build_mpo(wl.random_blocks(rng, 2, 2), 2, 0.1 + 0.2j, "V2")
    e0 = dense.boundary(W.shape[0])
    got = fit.mpo_overlap(bra, [W] * L, ket, e0, e0)
    ref = np.vdot(dense.mps_to_dense(bra), dense.dense_evolution_mpo(W, L) @ dense.mps_to_dense(ket))
    assert abs(got - ref) < 1e-12 * abs(ref)
