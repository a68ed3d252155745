"""Steps replayed from a captured HIP graph against steps issued launch by launch.

A step with use_graph runs uncaptured the first time its plan (shapes, options, buffers,
preconditioner state) is seen on a handle, is captured into a graph the second time and replayed
from the graph after that. The graph holds the same launches with the same arguments (only the
Jacobi and QR kernels go from cooperative to ordinary launches), so every step must reproduce the
uncaptured trajectory bit for bit -- site tensors, norms and discarded weights -- and stay on the
oracle's trajectory. Both handles keep the tile tuner off, so that they run the same tiles.
"""
import numpy as np
import pytest

from gpu_helpers import mpo_pair, say
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


def _normalise(ms):
    n = ofit.norm(ms)
    out = [m.copy() for m in ms]
    out[0] = out[0] / n
    return out


def _same(a, b):
    return all(x.shape == y.shape and np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("nsites", [2, 1], ids=["two-site", "one-site"])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_graph_replay_bitwise(mp, prec, nsites):
    L, D, steps = 12, 8, 6
    say("graph replay L=12 D=8", "fp64" if prec == 0 else "fp32", f"nsites={nsites}")
    rng = np.random.default_rng(41)
    psi = _normalise(wl.random_mps(rng, L, 2, D))
    W, Wo = mpo_pair(mp, wl.tfim(1.5), 2, -0.1j)
    hg, hp = mp.Handle(0), mp.Handle(0)
    try:
        for h in (hg, hp):
            h.set_tuning(mp.TUNE_OFF)
        dw = mp.DeviceMPO([W] * L)
        g = mp.DeviceMPS(psi, Dmax=D)
        p = mp.DeviceMPS(psi, Dmax=D)
        ref = psi
        uses = []
        for s in range(steps):
            sg = mp.step(hg, g, dw, prec=prec, input_right_canonical=s > 0, nsites=nsites, use_graph=True)
            sp = mp.step(hp, p, dw, prec=prec, input_right_canonical=s > 0, nsites=nsites)
            a, b = g.to_numpy(), p.to_numpy()
            uses.append(sg.graph)
            print(f"  step {s}: graph {sg.graph} norm {sg.norm:.15f} bonds {max(g.bond)}", flush=True)
            assert sp.graph == 0
            assert _same(a, b), s
            assert sg.norm == sp.norm and sg.discarded_sum == sp.discarded_sum, s
            assert g.bond == p.bond
            if nsites == 2:
                ref, _ = ofit.fit_step(ref, Wo, Dmax=D, nsweeps=2)
            else:
                ref, _ = ofit.fit_step_one_site(ref, Wo, nsweeps=2)
            assert 1 - abs(ofit.overlap(a, ref)) ** 2 < (1e-10 if prec == 0 else 1e-8), s
        torch.cuda.synchronize()
        # step 0 and the first canonical step run uncaptured, a later one is captured, and the
        # ones after it replay the graph
        assert uses[0] == 0 and 1 in uses and uses[-1] == 2, uses
    finally:
        hg.close()
        hp.close()


def test_graph_not_used_with_profile(mp):
    say("graph option with profiling")
    rng = np.random.default_rng(5)
    psi = _normalise(wl.random_mps(rng, 8, 2, 4))
    W, _ = mpo_pair(mp, wl.tfim(1.0), 2, -0.1j)
    h = mp.Handle(0)
    try:
        dm = mp.DeviceMPS(psi, Dmax=4)
        dw = mp.DeviceMPO([W] * 8)
        for s in range(3):
            st = mp.step(h, dm, dw, prec=1, input_right_canonical=s > 0, use_graph=True, profile=True)
            assert st.graph == 0 and st.profile["n_jacobi"] == st.visits
    finally:
        h.close()


def test_graph_batched_chains_bitwise(mp):
    """step_batched with use_graph: every chain captures and replays its own graph on its worker
    stream while the other workers run and synchronise their own steps; the chains match the
    uncaptured batched steps bit for bit."""
    say("graph replay step_batched, 12 chains")
    W, _ = mpo_pair(mp, wl.tfim(1.2), 2, -0.1j)
    shapes = [(10, 8), (12, 8), (9, 4), (14, 16), (8, 8), (11, 4), (16, 16), (10, 16), (13, 8), (9, 8),
              (12, 4), (15, 8)]
    hg, hp = mp.Handle(0), mp.Handle(0)
    try:
        G, P, M = [], [], []
        for k, (L, D) in enumerate(shapes):
            psi = _normalise(wl.random_mps(np.random.default_rng(60 + k), L, 2, D))
            G.append(mp.DeviceMPS(psi, Dmax=D))
            P.append(mp.DeviceMPS(psi, Dmax=D))
            M.append(mp.DeviceMPO([W] * L))
        wsg = mp.step_batched_workspace(G, M, mp.FP32)
        wsp = mp.step_batched_workspace(P, M, mp.FP32)
        last = None
        for s in range(5):
            sg = mp.step_batched(hg, G, M, prec=mp.FP32, input_right_canonical=s > 0, workspace=wsg,
                                 use_graph=True)
            sp = mp.step_batched(hp, P, M, prec=mp.FP32, input_right_canonical=s > 0, workspace=wsp)
            last = [x.graph for x in sg]
            print(f"  step {s}: graph {last}", flush=True)
            for c in range(len(shapes)):
                assert _same(G[c].to_numpy(), P[c].to_numpy()), (s, c)
                assert sg[c].norm == sp[c].norm, (s, c)
        assert all(u == 2 for u in last), last
    finally:
        hg.close()
        hp.close()
