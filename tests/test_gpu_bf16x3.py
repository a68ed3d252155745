"""GPU parity of the split-BF16x3 contraction mode (MPOEVO_BF16X3) against the CPU oracle.

The mode takes complex64 operands like the FP32 path. Each float is split into a bf16 head
h = bf16(x) and a bf16 tail t = bf16(x - h). Both roundings are to nearest with bf16's 8-bit
significand, so |x - h - t| <= 2^-16 |x|. The products h h + h t + t h are accumulated in float
and the t t term is dropped (at most 2^-16 |x y|). Every real product therefore carries about
3 * 2^-16 ~ 4.6e-5 relative error at worst. These errors have independent signs, so the norm-wise
error of a product stays near 2^-16 * O(1), whatever K is. A contraction chains at most three
products (environment times site, times W, times the bra or the other block), which gives the
tolerances below:
  contractions: element-wise error <= 2e-4 of the largest oracle entry, and relative Frobenius
                error <= 2e-4 (and, as a sanity check on the mode, >= 1e-9: the result is not an
                FP64 product);
  time step:    infidelity against the oracle step from the same input <= 1e-7 (the state error
                is ~1e-5 relative and enters the infidelity squared); norm within 1e-4 relative.
"""
import numpy as np
import pytest

from gpu_helpers import assert_close, mpo_pair
from oracle import fit as ofit
from paper_2302_14181_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL_CONTRACT = 2e-4


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


def _dev64(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to(torch.complex64).cuda()


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _cn(rng, *shape):
    return wl.complex_normal(rng, shape)


ENV_CASES = [  # Dbra_l, Dket_l, Dbra_r, Dket_r, d, w_l, w_r
    (1, 1, 2, 2, 2, 3, 3),
    (37, 45, 29, 33, 2, 3, 3),          # ragged tiles
    (130, 130, 130, 130, 2, 6, 6),      # several tiles, ragged tail
    (256, 256, 256, 256, 2, 8, 8),      # the D = 256 environment shape
    (20, 17, 23, 19, 2, 271, 271),      # long MPO bonds: the W contraction as a product
    (500, 237, 180, 300, 2, 4, 5),      # several stages with a ragged last one, split K
]


@pytest.mark.parametrize("side", ["left", "right"])
@pytest.mark.parametrize("dims", ENV_CASES, ids=[str(c) for c in ENV_CASES])
def test_env_update_bf16x3(mp, handle, dims, side):
    Dbl, Dkl, Dbr, Dkr, d, wl_, wr = dims
    rng = np.random.default_rng(3 + sum(dims))
    _say("env_update bf16x3", side, dims)
    bra, ket, W = _cn(rng, Dbl, d, Dbr), _cn(rng, Dkl, d, Dkr), _cn(rng, wl_, d, d, wr)
    if side == "left":
        E = _cn(rng, Dbl, wl_, Dkl)
        ref = ofit.env_left(E, bra, W, ket)
        out = torch.zeros((Dbr, wr, Dkr), dtype=torch.complex64, device="cuda")
        mp.env_update(handle, mp.LEFT, _dev64(E), _dev64(bra), _dev64(W), _dev64(ket), out, prec=mp.BF16X3)
    else:
        E = _cn(rng, Dbr, wr, Dkr)
        ref = ofit.env_right(E, bra, W, ket)
        out = torch.zeros((Dbl, wl_, Dkl), dtype=torch.complex64, device="cuda")
        mp.env_update(handle, mp.RIGHT, _dev64(E), _dev64(bra), _dev64(W), _dev64(ket), out, prec=mp.BF16X3)
    torch.cuda.synchronize()
    _, err = assert_close(out.cpu().numpy(), ref, TOL_CONTRACT, "env_update bf16x3")
    assert err > 1e-9, err


LA_CASES = [  # Dbra_l, Dket_l, Dket_m, Dket_r, Dbra_r, d, w_l, w_m, w_r
    (1, 1, 2, 4, 4, 2, 3, 3, 3),
    (33, 40, 47, 29, 35, 2, 3, 3, 3),
    (64, 64, 64, 64, 64, 2, 6, 6, 6),
    (10, 12, 14, 11, 9, 2, 271, 271, 271),
]


@pytest.mark.parametrize("dims", LA_CASES, ids=[str(c) for c in LA_CASES])
def test_local_apply_bf16x3(mp, handle, dims):
    Dbl, Dkl, Dkm, Dkr, Dbr, d, wl_, wm, wr = dims
    rng = np.random.default_rng(11 + sum(dims))
    _say("local_apply bf16x3", dims)
    L = _cn(rng, Dbl, wl_, Dkl)
    M1, M2 = _cn(rng, Dkl, d, Dkm), _cn(rng, Dkm, d, Dkr)
    W1, W2 = _cn(rng, wl_, d, d, wm), _cn(rng, wm, d, d, wr)
    R = _cn(rng, Dbr, wr, Dkr)
    ref = ofit.theta_two_site(L, M1, W1, M2, W2, R).reshape(Dbl * d, d * Dbr)
    th = torch.zeros((Dbl * d, d * Dbr), dtype=torch.complex128, device="cuda")
    mp.local_apply(handle, _dev64(L), _dev64(W1), _dev64(W2), _dev64(M1), _dev64(M2), _dev64(R), th,
                   prec=mp.BF16X3)
    torch.cuda.synchronize()
    _, err = assert_close(th.cpu().numpy(), ref, TOL_CONTRACT, "local_apply bf16x3")
    assert err > 1e-9, err


def test_bf16x3_needs_complex64(mp, handle):
    _say("bf16x3 dtype check")
    E = torch.zeros((2, 3, 2), dtype=torch.complex128, device="cuda")
    site = torch.zeros((2, 2, 2), dtype=torch.complex128, device="cuda")
    W = torch.zeros((3, 2, 2, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(mp.MpoevoError):
        mp.env_update(handle, mp.LEFT, E, site, W, site, E.clone(), prec=mp.BF16X3)


def _normalise(ms):
    n = ofit.norm(ms)
    out = [m.copy() for m in ms]
    out[0] = out[0] / n
    return out


@pytest.mark.parametrize("case", [(6, 4, 2, 8), (12, 8, 2, 24)], ids=str)
def test_step_bf16x3_random_state(mp, handle, case):
    L, D0, N, D = case
    _say("step bf16x3 random", case)
    rng = np.random.default_rng(L * 7 + D)
    psi = _normalise(wl.random_mps(rng, L, 2, D0))
    W, Wo = mpo_pair(mp, wl.tfim(1.0), N, -0.1j)
    ref, rst = ofit.fit_step(psi, Wo, Dmax=D, nsweeps=2)
    dm = mp.DeviceMPS(psi, Dmax=D)
    dw = mp.DeviceMPO([W] * L)
    st = mp.step(handle, dm, dw, nsweeps=2, prec=mp.BF16X3)
    out = dm.to_numpy()
    infid = 1 - abs(ofit.overlap(out, ref)) ** 2
    print(f"  infidelity {infid:.3e}", flush=True)
    assert infid < 1e-7, infid
    assert abs(st.norm - rst["norm"]) < 1e-4 * rst["norm"]
    assert abs(ofit.norm(out) - 1) < 1e-12


def test_step_bf16x3_long_range_order3_d64(mp, handle):
    """Split-BF16x3 step with the order-3 long-range MPO (w = 271) at L = 14, D = 64: the products
    take the bf16x3 128 x 64 tile. Against the oracle's fit from the same random state."""
    import json
    import os
    L, D = 14, 64
    _say("step bf16x3 long-range order 3 L=14 D=64")
    plan = handle.product_plan(mp.BF16X3, D * 271, 2 * D, D)
    print("  plan of the E ket product:", plan, flush=True)
    assert plan["tile"] == (128, 64)
    fit = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lr_fit_K6.json")))
    H = wl.lr_ising(np.array(fit["coeffs"]), np.array(fit["lambdas"]), 1.0)
    W, Wo = mpo_pair(mp, H, 3, -0.1j)
    psi = _normalise(wl.random_mps(np.random.default_rng(1464), L, 2, D))
    ref, rst = ofit.fit_step(psi, Wo, Dmax=D, nsweeps=2)
    dm = mp.DeviceMPS(psi, Dmax=D)
    st = mp.step(handle, dm, mp.DeviceMPO([W] * L), nsweeps=2, prec=mp.BF16X3)
    infid = 1 - abs(ofit.overlap(dm.to_numpy(), ref)) ** 2
    print(f"  infidelity {infid:.3e}", flush=True)
    assert infid < 1e-7, infid
    assert abs(st.norm - rst["norm"]) < 1e-4 * rst["norm"]
