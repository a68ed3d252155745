"""env_update_noalloc (the allocation-free variant of env_update, scratch in the library's
per-device static array) against env_update with a caller workspace, through the C ABI.

Two calls in a row per precision and side, the second with a smaller input (the array keeps the
first call's contents), each compared element-wise with env_update on the same inputs at the
contraction tolerance of the parity tests (FP64 1e-12, FP32 2e-5 of the largest entry), and with
the oracle. Dimensions beyond the array are rejected before any GPU work.
"""
import numpy as np
import pytest

from gpu_helpers import assert_close, say
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


# first the D = 256, w = 8 environment shape, then a smaller ragged one
CASES = [(256, 256, 256, 256, 2, 8, 8), (100, 131, 140, 77, 3, 4, 5)]


@pytest.mark.parametrize("prec", [1, 0], ids=["fp32", "fp64"])
@pytest.mark.parametrize("side", [0, 1], ids=["left", "right"])
def test_noalloc_matches_env_update_two_calls(mp, handle, prec, side):
    f64 = prec == mp.FP64
    dt = torch.complex128 if f64 else torch.complex64
    tol = 1e-12 if f64 else 2e-5
    for call, dims in enumerate(CASES):
        say("env_update_noalloc", "fp64" if f64 else "fp32", "left" if side == 0 else "right", "call", call, dims)
        Dbl, Dkl, Dbr, Dkr, d, wl_, wr = dims
        rng = np.random.default_rng(900 + 10 * call + 2 * side + prec)
        cn = lambda *s: wl.complex_normal(rng, s)  # noqa: E731
        bra, ket, W = cn(Dbl, d, Dbr), cn(Dkl, d, Dkr), cn(wl_, d, d, wr)
        if side == mp.LEFT:
            E = cn(Dbl, wl_, Dkl)
            ref = ofit.env_left(E, bra, W, ket)
        else:
            E = cn(Dbr, wr, Dkr)
            ref = ofit.env_right(E, bra, W, ket)
        t = {k: torch.from_numpy(v).to(dt).cuda() for k, v in dict(E=E, bra=bra, W=W, ket=ket).items()}
        a = torch.zeros(ref.shape, dtype=dt, device="cuda")
        b = torch.full(ref.shape, float("nan"), dtype=dt, device="cuda")
        mp.env_update(handle, side, t["E"], t["bra"], t["W"], t["ket"], a)
        mp.env_update_noalloc(handle, side, t["E"], t["bra"], t["W"], t["ket"], b)
        torch.cuda.synchronize()
        got, want = b.cpu().numpy(), a.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert_close(got, want, tol, "noalloc vs env_update")
        assert_close(got, ref, tol, "noalloc vs oracle")


def test_noalloc_rejects_oversized_dimensions(mp, handle):
    say("env_update_noalloc oversized dimensions (host-side rejection)")
    dims = [1024, 1024, 1024, 1024, 2, 8, 8]  # the intermediates alone need 256 MiB in FP32
    E = torch.zeros(8, dtype=torch.complex64, device="cuda")  # never read: rejected on the host
    p = mp._ptr(E)
    rc = mp.load().env_update_noalloc(handle.ptr, mp.LEFT, mp.FP32, p, p, p, p, p, mp._iarr(dims), None)
    assert rc == mp.ENOMEM, rc
    assert b"scratch" in mp.load().mpoevo_last_error(handle.ptr)
