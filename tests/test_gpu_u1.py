"""GPU parity of the U(1) two-site fit (sector tables through the C ABI) against the block-sparse
oracle (oracle/u1.py: dictionaries of blocks, per-charge SVDs, global top-D), on the XXZ chain
(Sec. 2.4) with seeded random U(1) states laid out densely in charge order.

Compared: the gauge-invariant overlap of the device result with the oracle's (infidelity <= 1e-12
FP64 / 1e-9 FP32, as for the dense step), the fitted norm, the discarded weight, and the charge
content of every new bond (the number of kept indices per charge, which the global top-D selection
fixes exactly when no singular values tie across blocks).
"""
import numpy as np
import pytest

from gpu_helpers import say
from oracle import fit as ofit, mpo as ompo, u1
from paper_2302_14181_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mp():
    from paper_2302_14181_amd import mpoevo
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mpoevo.load()
    return mpoevo


@pytest.fixture(scope="module")
def handle(mp):
    h = mp.Handle(0)
    yield h
    h.close()


def _case(mp, L, n_up, D0, seed, tau=-0.1j):
    H = wl.xxz(0.5)
    qp = H.phys_charge
    W, lc_lib = mp.mpo_build(H.A, H.B, H.C, H.Dloc, 2, tau, mp.V2_EXTENDED, H.inner_charge, qp)
    Wo = ompo.build_mpo(H, 2, tau, "V2")
    lc = ompo.level_charges(H, 2, tau, "V2")
    assert np.array_equal(lc_lib, lc)
    tables = wl.u1_sector_tables(L, n_up, D0, nsec=7, seed=seed)
    psi = wl.random_u1_mps(np.random.default_rng(seed), tables, qp)
    return qp, W, Wo, lc, tables, psi


def _charge_counts(charges):
    out = {}
    for q in charges:
        out[q] = out.get(q, 0) + 1
    return out


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", [(10, 5, 8, 8), (14, 7, 20, 20)], ids=str)
def test_u1_steps_against_block_oracle(mp, handle, case, prec):
    L, n_up, D0, D = case
    say("U(1) XXZ steps", case, "fp64" if prec == 0 else "fp32")
    qp, W, Wo, lc, tables, psi = _case(mp, L, n_up, D0, seed=L)
    dense, charges = wl.u1_dense(psi, tables, qp)
    dm = mp.DeviceMPS(dense, Dmax=D, charges=charges, phys_charge=qp)
    dw = mp.DeviceMPO([W] * L)
    ref, rbonds = psi, tables
    for k in range(2):
        ref, rbonds, rst = u1.fit_step(ref, rbonds, Wo, lc, qp, Dmax=D)
        st = mp.step(handle, dm, dw, prec=prec, input_right_canonical=k > 0)
        out = dm.to_numpy()
        refd = u1.to_dense(ref, rbonds, qp)
        infid = 1 - abs(ofit.overlap(out, refd)) ** 2
        print(f"  step {k}: infidelity {infid:.3e} norm {st.norm:.14f} vs {rst['norm']:.14f} "
              f"bonds {max(dm.bond)}", flush=True)
        assert infid < (1e-12 if prec == 0 else 1e-9), (k, infid)
        assert abs(st.norm - rst["norm"]) < (1e-10 if prec == 0 else 1e-6) * rst["norm"]
        assert abs(st.discarded_sum - sum(rst["discarded"])) < (1e-12 if prec == 0 else 1e-8)
        for b in range(L + 1):
            assert _charge_counts(dm.charges[b]) == {q: n for q, n in rbonds[b].items() if n > 0}, b
            assert dm.charges[b] == sorted(dm.charges[b])
    assert max(rst["discarded"]) > 1e-10  # the case truncates


def test_u1_step_conserves_charge_exactly(mp, handle):
    """The blocks outside the charge rule stay exactly zero on the device (FP32 path)."""
    L, n_up, D = 12, 6, 12
    say("U(1) charge rule on the device")
    qp, W, Wo, lc, tables, psi = _case(mp, L, n_up, 12, seed=5)
    dense, charges = wl.u1_dense(psi, tables, qp)
    dm = mp.DeviceMPS(dense, Dmax=D, charges=charges, phys_charge=qp)
    mp.step(handle, dm, mp.DeviceMPO([W] * L), prec=mp.FP32)
    out = dm.to_numpy()
    for i, M in enumerate(out):
        ql, qr = np.array(dm.charges[i]), np.array(dm.charges[i + 1])
        forbidden = ql[:, None, None] + np.array(qp)[None, :, None] != qr[None, None, :]
        assert np.all(M[forbidden] == 0), i


def test_u1_rejects_one_site(mp, handle):
    say("U(1) one-site request")
    qp, W, Wo, lc, tables, psi = _case(mp, 8, 4, 8, seed=2)
    dense, charges = wl.u1_dense(psi, tables, qp)
    dm = mp.DeviceMPS(dense, Dmax=8, charges=charges, phys_charge=qp)
    with pytest.raises(mp.MpoevoError) as e:
        mp.step(handle, dm, mp.DeviceMPO([W] * 8), nsites=1)
    assert e.value.code == mp.EUNSUPPORTED
