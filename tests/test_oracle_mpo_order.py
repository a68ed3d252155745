"""Pins of the oracle's order-N MPO against facts that do not come from its own formulas:
the bond-dimension table (Sec. 8.3), the error law of the order-N operator (Sec. 8.1: error
of order tau^(N+1) per step), closed forms (on-site only Hamiltonian, tau = 0), the exactness
of Alg. 2 (Sec. 4) and U(1) charge conservation."""
import numpy as np
import pytest

from oracle import dense, mpo
from paper_2302_14181_amd import workloads as wl

# Printed bond-dimension table of Sec. 8.3: coefficients of chi^0, chi^1, ...
PRINTED_DIMS = {1: [1, 1], 2: [1, 1, 1], 3: [1, 3, 1, 1], 4: [1, 5, 4, 1, 1]}


def _poly(coeffs, chi):
    return sum(c * chi ** p for p, c in enumerate(coeffs))


@pytest.mark.parametrize("chi", [1, 2, 3])
@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_bond_dimension_table(N, chi):
    H = wl.random_blocks(np.random.default_rng(N * 10 + chi), 2, chi)
    W = mpo.build_mpo(H, N, 0.1, "V2")
    assert W.shape[0] == W.shape[3] == _poly(PRINTED_DIMS[N], chi)


def test_v1_level_count():
    """V1 keeps the Alg. 2 representatives; enumerated independently here: all tuples with a 2,
    canonicalised (1s to the front if n3 <= n1, else 3s to the back), plus (1,...,1)."""
    import itertools
    for N in (1, 2, 3, 4):
        reps = {(1,) * N}
        for t in itertools.product((1, 2, 3), repeat=N):
            if 2 not in t:
                continue
            if t.count(3) <= t.count(1):
                s = tuple(sorted(t, key=lambda x: 0 if x == 1 else 1))
            else:
                s = tuple(sorted(t, key=lambda x: 1 if x == 3 else 0))
            reps.add(s)
        for chi in (1, 2):
            H = wl.random_blocks(np.random.default_rng(3), 2, chi)
            W = mpo.build_mpo(H, N, 0.1, "V1")
            assert W.shape[0] == sum(chi ** r.count(2) for r in reps)


def _err(H, N, tau, variant, L):
    Hd = dense.dense_hamiltonian(mpo.hamiltonian_mpo(H), L)
    U = dense.expm(tau, Hd)
    Wd = dense.dense_evolution_mpo(mpo.build_mpo(H, N, tau, variant), L)
    return np.linalg.norm(Wd - U, 2)


@pytest.mark.parametrize("variant", ["V1", "V2"])
@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_error_order_random_hamiltonian(N, variant):
    """Random non-Hermitian H (chi = 2), real tau: ||W_N(tau) - exp(tau H)|| ~ tau^(N+1)."""
    H = wl.random_blocks(np.random.default_rng(100 + N), 2, 2, a_scale=0.4)
    taus = [0.08, 0.04, 0.02]
    errs = [_err(H, N, t, variant, 5) for t in taus]
    slopes = [np.log(errs[i] / errs[i + 1]) / np.log(taus[i] / taus[i + 1]) for i in range(2)]
    assert min(slopes) >= N + 1 - 0.15, (errs, slopes)


@pytest.mark.parametrize("variant", ["V1", "V2"])
@pytest.mark.parametrize("N", [1, 2, 3])
def test_error_order_tfim_real_time(N, variant):
    """TFIM, tau = -i dt (unitary target): error slope at least N + 1 (the second-order V2
    operator may do better on this model, as Sec. 8.2 observes for the Ising cylinder)."""
    H = wl.tfim(1.0)
    dts = [0.1, 0.05, 0.025]
    errs = [_err(H, N, -1j * t, variant, 6) for t in dts]
    slopes = [np.log(errs[i] / errs[i + 1]) / np.log(dts[i] / dts[i + 1]) for i in range(2)]
    assert min(slopes) >= N + 1 - 0.15, (errs, slopes)


def _taylor(X, M):
    out = np.eye(X.shape[0], dtype=np.complex128)
    term = np.eye(X.shape[0], dtype=np.complex128)
    for m in range(1, M + 1):
        term = term @ X / m
        out = out + term
    return out


@pytest.mark.parametrize("variant,extra", [("V1", 0), ("V2", 1)])
@pytest.mark.parametrize("N", [1, 2, 3])
def test_onsite_only_closed_form(N, variant, extra):
    """B = C = 0: the MPO is the product of the order-M Taylor polynomials of exp(tau Dloc),
    M = N (V1) or N + 1 (V2)."""
    rng = np.random.default_rng(7)
    H = wl.random_blocks(rng, 2, 1)
    H.B[:] = 0
    H.C[:] = 0
    tau = 0.3 - 0.2j
    L = 3
    Wd = dense.dense_evolution_mpo(mpo.build_mpo(H, N, tau, variant), L)
    T = _taylor(tau * H.Dloc, N + extra)
    ref = np.kron(np.kron(T, T), T)
    assert np.max(np.abs(Wd - ref)) < 1e-13


@pytest.mark.parametrize("variant", ["V1", "V2"])
def test_tau_zero_is_identity(variant):
    H = wl.random_blocks(np.random.default_rng(5), 2, 2)
    for N in (1, 2, 3):
        Wd = dense.dense_evolution_mpo(mpo.build_mpo(H, N, 0.0, variant), 4)
        assert np.max(np.abs(Wd - np.eye(16))) < 1e-14


@pytest.mark.parametrize("N", [2, 3])
def test_exact_compression_is_exact(N):
    """Alg. 2 leaves the contracted operator unchanged (V1, random H, chi = 2, L = 4)."""
    H = wl.random_blocks(np.random.default_rng(21), 2, 2)
    tau = 0.2 + 0.1j
    folded = mpo.fold(mpo.hamiltonian_power(H, N), tau)
    W_fold, _, _ = mpo.assemble(folded)
    W_comp, _, _ = mpo.assemble(mpo.exact_compress(folded))
    assert W_comp.shape[0] < W_fold.shape[0]
    a = dense.dense_evolution_mpo(W_fold, 4)
    b = dense.dense_evolution_mpo(W_comp, 4)
    assert np.max(np.abs(a - b)) < 1e-13 * max(1.0, np.max(np.abs(a)))


def test_hamiltonian_mpo_matches_pauli_sum():
    """The level-(1,2,3) MPO of the TFIM blocks contracts to -sum ZZ - g sum X (Sec. 2.4)."""
    L, g = 5, 0.7
    Hd = dense.dense_hamiltonian(mpo.hamiltonian_mpo(wl.tfim(g)), L)
    ref = np.zeros((2 ** L, 2 ** L), dtype=np.complex128)
    for i in range(L - 1):
        ref -= dense.local_op(wl.SZ, i, L) @ dense.local_op(wl.SZ, i + 1, L)
    for i in range(L):
        ref -= g * dense.local_op(wl.SX, i, L)
    assert np.max(np.abs(Hd - ref)) < 1e-13


def test_xxz_charge_conservation():
    """Every nonzero W[alpha, s', s, beta] of the order-2 XXZ MPO obeys
    q_alpha + q(s') = q(s) + q_beta, with the level charges of the builder."""
    H = wl.xxz(0.5)
    for N in (1, 2, 3):
        W = mpo.build_mpo(H, N, -0.1j, "V2")
        q = mpo.level_charges(H, N, -0.1j, "V2")
        qs = H.phys_charge
        nz = np.argwhere(np.abs(W) > 1e-15)
        assert len(nz) > 0
        for a, sp, s, b in nz:
            assert q[a] + qs[sp] == qs[s] + q[b]


def test_v2_more_precise_than_v1():
    """Sec. 8.1 observes that the extended and approximately compressed MPO is the more
    precise one; checked on the TFIM for orders 1-3 (soft claim of the paper)."""
    H = wl.tfim(1.0)
    for N in (1, 2, 3):
        e1 = _err(H, N, -0.1j, "V1", 6)
        e2 = _err(H, N, -0.1j, "V2", 6)
        assert e2 < e1, (N, e1, e2)


# ---- splitting composites (Sec. 8.3, splitting schemes)

def test_compose_is_the_operator_product():
    """The composed site tensor contracts to the dense product of the two dense operators (brute
    force on three sites, random tensors, boundary index 0 on both ends)."""
    rng = np.random.default_rng(11)
    Wa = wl.complex_normal(rng, (3, 2, 2, 3))
    Wb = wl.complex_normal(rng, (2, 2, 2, 2))
    L = 3
    A = dense.contract_mpo([Wa] * L, dense.boundary(3), dense.boundary(3))
    B = dense.contract_mpo([Wb] * L, dense.boundary(2), dense.boundary(2))
    C = dense.contract_mpo([mpo.compose(Wa, Wb)] * L, dense.boundary(6), dense.boundary(6))
    assert np.allclose(C, A @ B, atol=1e-12 * np.linalg.norm(A @ B))


def test_split_step_constants():
    """t1 + t2 = 1 and t1 t2 = 1/2: the composite's tau and tau^2 terms are those of exp."""
    assert abs(mpo.SPLIT_T1 + mpo.SPLIT_T2 - 1) < 1e-15
    assert abs(mpo.SPLIT_T1 * mpo.SPLIT_T2 - 0.5) < 1e-15


@pytest.mark.parametrize("chi", [1, 2, 3])
def test_split_composite_bond_exceeds_second_order_table(chi):
    """Sec. 8.3: the composite of first-order operators has bond (1 + chi)^2, larger than the
    printed second-order entry 1 + chi + chi^2 for every chi >= 1."""
    H = wl.random_blocks(np.random.default_rng(chi), 2, chi)
    Wc = mpo.split_composite(H, 0.1)
    assert Wc.shape[0] == Wc.shape[3] == (1 + chi) ** 2
    assert Wc.shape[0] > _poly(PRINTED_DIMS[2], chi) == mpo.build_mpo(H, 2, 0.1, "V2").shape[0]


def _err_split(H, tau, variant, L):
    Hd = dense.dense_hamiltonian(mpo.hamiltonian_mpo(H), L)
    U = dense.expm(tau, Hd)
    Wd = dense.dense_evolution_mpo(mpo.split_composite(H, tau, variant), L)
    return np.linalg.norm(Wd - U, 2)


@pytest.mark.parametrize("variant", ["V1", "V2"])
def test_split_composite_is_second_order(variant):
    """||O1(t1 tau) O1(t2 tau) - exp(tau H)|| ~ tau^3, against the exact exponential (TFIM real
    time and a random non-Hermitian H); the single first-order operator only reaches tau^2."""
    for H, L, taus in ((wl.tfim(1.0), 6, [-0.1j, -0.05j, -0.025j]),
                       (wl.random_blocks(np.random.default_rng(7), 2, 2, a_scale=0.4), 5, [0.1, 0.05, 0.025])):
        errs = [_err_split(H, t, variant, L) for t in taus]
        slopes = [np.log(errs[i] / errs[i + 1]) / np.log(2) for i in range(2)]
        assert min(slopes) >= 3 - 0.15, (errs, slopes)
        e1 = [_err(H, 1, t, variant, L) for t in taus[1:]]
        assert np.log(e1[0] / e1[1]) / np.log(2) < 2.6
