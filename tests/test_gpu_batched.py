"""GPU tests of step_batched: independent chains advanced concurrently.

Each chain of a batch runs the same kernels as `step` on that chain alone, so the batched result
must equal the one-by-one result (to 1e-12 element-wise: the same arithmetic in the same order),
and through it the oracle's step (infidelity <= 1e-12 FP64 / 1e-9 FP32, as for `step`).
"""
import numpy as np
import pytest

from gpu_helpers import mpo_pair
from oracle import fit as ofit
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


def _say(*a):
    print("[case]", *a, flush=True)


def _normalise(ms):
    n = ofit.norm(ms)
    out = [m.copy() for m in ms]
    out[0] = out[0] / n
    return out


# (g, L, D0, D): uneven chains (lengths, bond dimensions, couplings)
CHAINS = [(0.7, 6, 4, 8), (1.3, 9, 6, 16), (1.0, 12, 8, 12), (0.55, 7, 3, 6), (1.45, 10, 5, 20),
          (0.9, 8, 8, 8), (1.2, 5, 2, 4), (0.6, 11, 6, 10), (1.1, 13, 4, 14), (0.8, 6, 5, 24)]


def _inputs(mp, chains, seed, oracle_mpos=False):
    """Random states and the chains' MPOs (device side; with oracle_mpos also the oracle's own)."""
    rng = np.random.default_rng(seed)
    psis, Ws, Wos = [], [], []
    for g, L, D0, _ in chains:
        psis.append(_normalise(wl.random_mps(rng, L, 2, D0)))
        W, Wo = mpo_pair(mp, wl.tfim(g), 2, -0.1j)
        Ws.append(W)
        Wos.append(Wo)
    return (psis, Ws, Wos) if oracle_mpos else (psis, Ws)


def _max_diff(a, b):
    assert [x.shape for x in a] == [y.shape for y in b]
    return max(float(np.max(np.abs(x - y))) for x, y in zip(a, b))


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_batched_equals_one_by_one_and_oracle(mp, handle, prec):
    chains = CHAINS[:6]
    _say("step_batched", len(chains), "chains", "fp64" if prec == 0 else "fp32")
    psis, Ws, Wos = _inputs(mp, chains, 41, oracle_mpos=True)
    dms = [mp.DeviceMPS(p, Dmax=c[3]) for p, c in zip(psis, chains)]
    dws = [mp.DeviceMPO([W] * c[1]) for W, c in zip(Ws, chains)]
    stats = mp.step_batched(handle, dms, dws, nsweeps=2, prec=prec)
    for c, (chain, psi, W) in enumerate(zip(chains, psis, Ws)):
        one = mp.DeviceMPS(psi, Dmax=chain[3])
        st1 = mp.step(handle, one, mp.DeviceMPO([W] * chain[1]), nsweeps=2, prec=prec)
        out_b, out_1 = dms[c].to_numpy(), one.to_numpy()
        assert dms[c].bond == one.bond, c
        diff = _max_diff(out_b, out_1)
        assert diff <= 1e-12, (c, diff)
        assert abs(stats[c].norm - st1.norm) <= 1e-12 * st1.norm
        assert stats[c].visits == 4 * (chain[1] - 1)
        if c < 3:  # the oracle on the first chains
            ref, rst = ofit.fit_step(psi, Wos[c], Dmax=chain[3], nsweeps=2)
            infid = 1 - abs(ofit.overlap(out_b, ref)) ** 2
            assert infid < (1e-12 if prec == 0 else 1e-9), (c, infid)


def test_batched_more_chains_than_streams_two_steps(mp, handle):
    """Ten chains (more than the worker streams), two consecutive steps on one workspace (the
    per-chain truncation preconditioners carry over), against two one-by-one steps per chain."""
    _say("step_batched 10 chains x 2 steps fp64")
    psis, Ws = _inputs(mp, CHAINS, 43)
    dms = [mp.DeviceMPS(p, Dmax=c[3]) for p, c in zip(psis, CHAINS)]
    dws = [mp.DeviceMPO([W] * c[1]) for W, c in zip(Ws, CHAINS)]
    ws = mp.step_batched_workspace(dms, dws, mp.FP64)
    mp.step_batched(handle, dms, dws, workspace=ws)
    mp.step_batched(handle, dms, dws, workspace=ws, input_right_canonical=True)
    for c, (chain, psi, W) in enumerate(zip(CHAINS, psis, Ws)):
        one = mp.DeviceMPS(psi, Dmax=chain[3])
        dw = mp.DeviceMPO([W] * chain[1])
        ws1 = mp.step_workspace(one, dw, mp.FP64)
        mp.step(handle, one, dw, workspace=ws1)
        mp.step(handle, one, dw, workspace=ws1, input_right_canonical=True)
        out_b, out_1 = dms[c].to_numpy(), one.to_numpy()
        assert dms[c].bond == one.bond, c
        infid = 1 - abs(ofit.overlap(out_b, out_1)) ** 2
        assert infid < 1e-13, (c, infid)


def test_batched_rejects_shared_chains(mp, handle):
    _say("step_batched argument errors")
    psis, Ws = _inputs(mp, CHAINS[:1], 45)
    dm = mp.DeviceMPS(psis[0], Dmax=CHAINS[0][3])
    dw = mp.DeviceMPO([Ws[0]] * CHAINS[0][1])
    with pytest.raises(mp.MpoevoError):
        mp.step_batched(handle, [dm, dm], [dw, dw])
    with pytest.raises(mp.MpoevoError):
        mp.step_batched(handle, [dm], [dw], nsweeps=0)
