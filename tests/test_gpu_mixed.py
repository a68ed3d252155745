"""GPU parity of the automatic mode's mixed sweep (one-site updates at sites whose two bonds are
frozen at their largest value, two-site updates elsewhere) against the oracle's fit_step_mixed:
states with some bonds still growing, FP64 and FP32 contractions, a short-range and the
long-range order-3 MPO; exactness at complete bonds against the dense W|psi>; the fallback to
two-site updates when a frozen bond shrinks; and bitwise replay from a captured graph.

Compared: the gauge-invariant infidelity of the two results (<= 1e-12 FP64, 1e-9 FP32, as for the
other step parity tests), the fitted norm, the discarded weights and the count of one-site visits.
"""
import json
import os

import numpy as np
import pytest

from gpu_helpers import mpo_pair, say
from oracle import dense, fit as ofit
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


def _normalise(ms):
    n = ofit.norm(ms)
    out = [m.copy() for m in ms]
    out[0] = out[0] / n
    return out


def _caps(L, D, d=2):
    return [min(D, d ** min(b, L - b)) for b in range(L + 1)]


def _check(mp, handle, psi, W, Wo, D, prec, right_canonical=False):
    ref, rst = ofit.fit_step_mixed(psi, Wo, D)
    dm = mp.DeviceMPS(psi, Dmax=D)
    st = mp.step(handle, dm, mp.DeviceMPO([W] * len(psi)), prec=prec, nsites=mp.NSITES_AUTO,
                 input_right_canonical=right_canonical)
    out = dm.to_numpy()
    infid = 1 - abs(ofit.overlap(out, ref)) ** 2
    n1 = rst["kinds"].count(1)
    print(f"  one-site visits {st.one_site_visits} (oracle {n1} of {len(rst['kinds'])}), redo {st.two_site_redo}, "
          f"infidelity {infid:.3e}, norm {st.norm:.14f} vs {rst['norm']:.14f}", flush=True)
    assert st.one_site_visits == n1 and st.two_site_redo == int(rst["fallback"])
    assert infid < (1e-12 if prec == 0 else 1e-9), infid
    assert abs(st.norm - rst["norm"]) < (1e-10 if prec == 0 else 1e-6) * rst["norm"]
    assert abs(st.discarded_max - max(rst["discarded"])) < (1e-12 if prec == 0 else 1e-8)
    assert dm.bond == rst["bond_dims"]
    return st, rst


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", [(12, 8, (5, 6)), (14, 16, (4, 9, 10)), (10, 8, (2,)), (9, 4, (7,))], ids=str)
def test_mixed_step_parity(mp, handle, case, prec):
    """(L, Dmax, bonds below their largest value); the rest at min(Dmax, 2^b, 2^(L-b))."""
    L, D, growing = case
    say("mixed step TFIM", case, "fp64" if prec == 0 else "fp32")
    dims = _caps(L, D)
    for b in growing:
        dims[b] = max(1, dims[b] - 2)
    rng = np.random.default_rng(500 + L + D)
    psi = _normalise(wl.random_mps(rng, L, 2, D, dims))
    W, Wo = mpo_pair(mp, wl.tfim(1.3), 2, -0.12j)
    st, rst = _check(mp, handle, psi, W, Wo, D, prec)
    assert 0 < st.one_site_visits < st.visits


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_mixed_step_long_range_order3(mp, handle, prec):
    """w = 271, L = 10, Dmax = 16: bonds 4 and 5 growing."""
    say("mixed step long-range order 3 w=271 L=10 D=16", "fp64" if prec == 0 else "fp32")
    fit = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lr_fit_K6.json")))
    H = wl.lr_ising(np.array(fit["coeffs"]), np.array(fit["lambdas"]), 1.0)
    W, Wo = mpo_pair(mp, H, 3, -0.1j)
    assert W.shape[0] == 271
    L, D = 10, 16
    dims = _caps(L, D)
    dims[4], dims[5] = 12, 13
    psi = _normalise(wl.random_mps(np.random.default_rng(77), L, 2, D, dims))
    _check(mp, handle, psi, W, Wo, D, prec)


def test_mixed_step_complete_bonds_exact(mp, handle):
    say("mixed step at complete bonds, against the dense W psi")
    L, D = 8, 16
    dims = [1, 2, 4, 8, 9, 8, 4, 2, 1]
    rng = np.random.default_rng(81)
    psi = _normalise(wl.random_mps(rng, L, 2, D, dims))
    W, Wo = mpo_pair(mp, wl.tfim(0.9), 3, 0.05 - 0.08j)
    v = dense.dense_evolution_mpo(Wo, L) @ dense.mps_to_dense(psi)
    dm = mp.DeviceMPS(psi, Dmax=D)
    st = mp.step(handle, dm, mp.DeviceMPO([W] * L), prec=mp.FP64, nsites=mp.NSITES_AUTO)
    f = dense.mps_to_dense(dm.to_numpy())
    assert st.one_site_visits > 0
    assert abs(st.norm - np.linalg.norm(v)) < 1e-12 * np.linalg.norm(v)
    assert 1 - abs(np.vdot(f, v)) ** 2 / np.linalg.norm(v) ** 2 < 1e-12


def test_mixed_step_falls_back_when_a_frozen_bond_shrinks(mp, handle):
    """Bond 1 is at its largest value (2) but the state is a product there: the two-site update of
    that bond keeps one value, and the step is redone with two-site updates (as the oracle does).
    FP64 only: with FP32 contractions the vanishing singular value comes out at the rounding of
    the products (about 1e-7 of the largest), above the cutoff, so the bond keeps two values."""
    say("mixed step fallback")
    rng = np.random.default_rng(9)
    L, D = 6, 4
    psi = wl.random_mps(rng, L, 2, D, [1, 2, 3, 4, 4, 2, 1])
    psi[0] = np.zeros_like(psi[0])
    psi[0][0, :, 0] = [0.6, 0.8]
    psi = _normalise(psi)
    W, Wo = mpo_pair(mp, wl.tfim(1.0), 1, 0.0)
    st, rst = _check(mp, handle, psi, W, Wo, D, 0)
    assert st.two_site_redo == 1 and rst["fallback"]


def _reload(dm, sites):
    """The same input again in the same device buffers (so that the step's plan repeats)."""
    for t, s_ in zip(dm.buf, sites):
        flat = torch.from_numpy(np.ascontiguousarray(s_, dtype=np.complex128).reshape(-1))
        t.zero_()
        t[: flat.numel()].copy_(flat)
    dm.bond = [1] + [int(s_.shape[2]) for s_ in sites]


def test_mixed_step_graph_replay_bitwise(mp, handle):
    """The same mixed step repeated from the same buffers on two handles in lock-step (both carry
    the same preconditioner state from pass to pass), one with use_graph: once its plan repeats it
    is captured and then replayed, and every pass matches the other handle's launch-by-launch pass
    bit for bit."""
    say("mixed step graph replay")
    L, D = 12, 8
    dims = _caps(L, D)
    dims[6] = 5
    psi = ofit.right_canonicalize(_normalise(wl.random_mps(np.random.default_rng(31), L, 2, D, dims)))
    W, _ = mpo_pair(mp, wl.tfim(1.1), 2, -0.1j)
    hg, hp = mp.Handle(0), mp.Handle(0)
    try:
        for h in (hg, hp):
            h.set_tuning(mp.TUNE_OFF)
        dw = mp.DeviceMPO([W] * L)
        g, p = mp.DeviceMPS(psi, Dmax=D), mp.DeviceMPS(psi, Dmax=D)
        uses = []
        for k in range(6):
            _reload(g, psi)
            _reload(p, psi)
            sg = mp.step(hg, g, dw, prec=mp.FP32, nsites=mp.NSITES_AUTO, input_right_canonical=True,
                         use_graph=True)
            sp = mp.step(hp, p, dw, prec=mp.FP32, nsites=mp.NSITES_AUTO, input_right_canonical=True)
            uses.append(sg.graph)
            out, ref = g.to_numpy(), p.to_numpy()
            print(f"  pass {k + 1}: graph {sg.graph}, one-site visits {sg.one_site_visits}, norm {sg.norm!r}",
                  flush=True)
            assert sg.one_site_visits == sp.one_site_visits > 0 and sp.graph == 0
            assert all(np.array_equal(a, b) for a, b in zip(out, ref)) and sg.norm == sp.norm, k
        torch.cuda.synchronize()
        assert 1 in uses and uses[-1] == 2, uses
    finally:
        hg.close()
        hp.close()
