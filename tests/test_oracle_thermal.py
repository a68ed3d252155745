"""Pins of the oracle's finite-temperature path (purification on a finite chain; the counterpart of
the exp(-beta H) construction of Sec. 8.4): the purified operator and the beta = 0 state against
the closed form <O>_{beta=0} = Tr O / d^L, and the imaginary-time evolution by the order-N MPO
against the exact thermal energy Tr(H exp(-beta H)) / Tr exp(-beta H) of the dense Hamiltonian,
converging as delta^N in the step delta (orders 2 and 3)."""
import numpy as np
import pytest

from oracle import dense, fit as ofit, mpo
from paper_2302_14181_amd import workloads as wl


def test_purified_operator_at_infinite_temperature_is_the_normalised_trace():
    rng = np.random.default_rng(3)
    W = wl.complex_normal(rng, (3, 2, 2, 3))
    L = 3
    O = dense.contract_mpo([W] * L, dense.boundary(3), dense.boundary(3))
    Op = dense.contract_mpo([mpo.purify(W)] * L, dense.boundary(3), dense.boundary(3))
    v = dense.mps_to_dense(wl.infinite_temperature(L))
    assert abs(np.vdot(v, v) - 1) < 1e-14
    assert abs(np.vdot(v, Op @ v) - np.trace(O) / 2 ** L) < 1e-12 * max(1, abs(np.trace(O)))


def test_infinite_temperature_energy_of_a_hermitian_chain():
    H = wl.random_hermitian_blocks(np.random.default_rng(9), 2, 2)
    L = 5
    Hd = dense.dense_hamiltonian(mpo.hamiltonian_mpo(H), L)
    Hp = mpo.purify(mpo.hamiltonian_mpo(H))
    w = Hp.shape[0]
    e = ofit.mpo_expectation(wl.infinite_temperature(L), [Hp] * L, dense.boundary(w, 0), dense.boundary(w, w - 1))
    assert abs(np.trace(Hd)) > 1e-3
    assert abs(e - np.trace(Hd) / 2 ** L) < 1e-12 * abs(np.trace(Hd))


def _thermal_energy(H, N, delta, K, L, D):
    Hp = mpo.purify(mpo.hamiltonian_mpo(H))
    w = Hp.shape[0]
    W = mpo.purify(mpo.build_mpo(H, N, -delta, "V2"))
    s = wl.infinite_temperature(L)
    for _ in range(K):
        s, _ = ofit.fit_step(s, W, Dmax=D)
    return (ofit.mpo_expectation(s, [Hp] * L, dense.boundary(w, 0), dense.boundary(w, w - 1))
            / ofit.overlap(s, s)).real


def _exact_energy(H, beta, L):
    lam = np.linalg.eigvalsh(dense.dense_hamiltonian(mpo.hamiltonian_mpo(H), L))
    p = np.exp(-beta * (lam - lam.min()))
    return float((lam * p).sum() / p.sum())


@pytest.mark.parametrize("N", [2, 3])
def test_thermal_energy_converges_with_the_order(N):
    """TFIM (g = 1), L = 8, beta = 1 reached in K steps of exp(-delta H) (beta / 2 = K delta)."""
    H, L = wl.tfim(1.0), 8
    ex = _exact_energy(H, 1.0, L)
    errs = [abs(_thermal_energy(H, N, dl, K, L, 64) - ex) for dl, K in ((0.1, 5), (0.05, 10))]
    slope = np.log(errs[0] / errs[1]) / np.log(2)
    assert slope > N - 0.3, (errs, slope)
    assert errs[1] < (2e-3 if N == 2 else 1e-4), errs
