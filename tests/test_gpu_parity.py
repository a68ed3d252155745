"""GPU parity of the C ABI device calls against the CPU oracle (MI355X only).

Every case prints its name, seed and shape before touching the GPU. Tolerances:
  FP64 contractions: element-wise error <= 1e-12 of the largest oracle entry (and relative
            Frobenius error <= 1e-12);
  FP32 contractions: the same with 2e-5: three chained float products, each rounding its
            output (2^-24 relative) and summing K <= 2048 terms whose rounding errors add with
            random signs (about sqrt(K) 2^-24 of the summed magnitudes, a few 1e-7 of the largest
            output); the three-product complex form adds up to two such terms to Im;
  FP64 SVD: singular values to 1e-12 relative to sigma_1, factors orthonormal to 1e-12,
            the rank-k product equal to the optimal rank-k approximation to 1e-11.
  Time step (gauge-invariant): infidelity against the oracle step from the same input
            <= 1e-12 (FP64) / 1e-9 (FP32); |norm - oracle norm| <= 1e-10 (FP64) / 1e-6 (FP32)
            relative (the FP32 projection carries float rounding, ~1e-7 relative).
"""
import numpy as np
import pytest

from gpu_helpers import assert_close, mpo_pair, say
from oracle import dense, fit as ofit, mpo as ompo
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


_say = say


def _dev(x, prec64=True):
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128))
    if not prec64:
        t = t.to(torch.complex64)
    return t.cuda()


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _cn(rng, *shape):
    return wl.complex_normal(rng, shape)


ENV_CASES = [  # Dbra_l, Dket_l, Dbra_r, Dket_r, d, w_l, w_r
    (1, 1, 2, 2, 2, 3, 3),
    (37, 45, 29, 33, 2, 3, 3),
    (64, 64, 64, 64, 2, 8, 8),
    (100, 131, 140, 77, 3, 4, 5),
    (130, 130, 130, 130, 2, 6, 6),
    (20, 17, 23, 19, 2, 271, 271),  # the order-3 long-range Ising MPO bond: W contraction as a product
    (9, 11, 13, 10, 2, 13, 40),     # one short (register kernel) and one long MPO leg
    # FP32 left: E.ket on 64 x 64 tiles over several stages with a ragged last one (K = 237), the
    # bra product with K = 1000 split in two over 64-deep stages, a partial W output group
    (500, 237, 180, 300, 2, 4, 5),
]


@pytest.mark.parametrize("prec64", [True, False], ids=["fp64", "fp32"])
@pytest.mark.parametrize("side", ["left", "right"])
@pytest.mark.parametrize("dims", ENV_CASES, ids=[str(c) for c in ENV_CASES])
def test_env_update_parity(mp, handle, dims, side, prec64):
    Dbl, Dkl, Dbr, Dkr, d, wl_, wr = dims
    rng = np.random.default_rng(sum(dims))
    _say("env_update", side, "fp64" if prec64 else "fp32", dims)
    bra, ket, W = _cn(rng, Dbl, d, Dbr), _cn(rng, Dkl, d, Dkr), _cn(rng, wl_, d, d, wr)
    if side == "left":
        E = _cn(rng, Dbl, wl_, Dkl)
        ref = ofit.env_left(E, bra, W, ket)
        out = torch.zeros((Dbr, wr, Dkr), dtype=torch.complex128 if prec64 else torch.complex64, device="cuda")
        mp.env_update(handle, mp.LEFT, _dev(E, prec64), _dev(bra, prec64), _dev(W, prec64), _dev(ket, prec64), out)
    else:
        E = _cn(rng, Dbr, wr, Dkr)
        ref = ofit.env_right(E, bra, W, ket)
        out = torch.zeros((Dbl, wl_, Dkl), dtype=torch.complex128 if prec64 else torch.complex64, device="cuda")
        mp.env_update(handle, mp.RIGHT, _dev(E, prec64), _dev(bra, prec64), _dev(W, prec64), _dev(ket, prec64), out)
    torch.cuda.synchronize()
    assert_close(out.cpu().numpy(), ref, 1e-12 if prec64 else 2e-5, "env_update")


@pytest.mark.parametrize("prec64", [True, False], ids=["fp64", "fp32"])
def test_env_update_microbench_shape(mp, handle, prec64):
    """The D = 256, d = 2, w = 8 microbenchmark operands (seed 0), both sides; sampled full-size check."""
    _say("env_update microbench D=256 w=8", "fp64" if prec64 else "fp32")
    E, M, N, W = wl.env_microbench_inputs(0)
    ref = ofit.env_left(E, N, W, M)
    out = torch.zeros((256, 8, 256), dtype=torch.complex128 if prec64 else torch.complex64, device="cuda")
    mp.env_update(handle, mp.LEFT, _dev(E, prec64), _dev(N, prec64), _dev(W, prec64), _dev(M, prec64), out)
    torch.cuda.synchronize()
    assert_close(out.cpu().numpy(), ref, 1e-12 if prec64 else 2e-5, "left")
    ref = ofit.env_right(E, N, W, M)
    mp.env_update(handle, mp.RIGHT, _dev(E, prec64), _dev(N, prec64), _dev(W, prec64), _dev(M, prec64), out)
    torch.cuda.synchronize()
    assert_close(out.cpu().numpy(), ref, 1e-12 if prec64 else 2e-5, "right")


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp64", "fp32", "bf16x3"])
def test_env_update_large_bond_tiles(mp, handle, prec):
    """D = 64, w = 271 (the order-3 long-range MPO bond): the W contraction runs as batched
    products of 542 x 64 outputs over 64 batches, which the planner puts on the 128 x 64 tile
    (5 x 1 x 64 = 320 workgroups; the 128 x 128 tile would be half empty at 64 columns). Both
    sides, element-wise against the oracle."""
    dims = (64, 64, 64, 64, 2, 271, 271)
    _say("env_update large-bond tile", dims, ["fp64", "fp32", "bf16x3"][prec])
    plan = handle.product_plan(prec, 2 * 271, 64, 2 * 271, 64)
    print("  plan of the W contraction product:", plan, flush=True)
    if prec != mp.FP64:
        assert plan["tile"] == (128, 64) and plan["splits"] == 1
    rng = np.random.default_rng(271)
    Dbl, Dkl, Dbr, Dkr, d, wl_, wr = dims
    bra, ket, W = _cn(rng, Dbl, d, Dbr), _cn(rng, Dkl, d, Dkr), _cn(rng, wl_, d, d, wr)
    E = _cn(rng, Dbl, wl_, Dkl)
    f64 = prec == mp.FP64
    tol = {0: 1e-12, 1: 2e-5, 2: 2e-4}[prec]
    for side, ref in ((mp.LEFT, ofit.env_left(E, bra, W, ket)), (mp.RIGHT, ofit.env_right(E, bra, W, ket))):
        out = torch.zeros(ref.shape, dtype=torch.complex128 if f64 else torch.complex64, device="cuda")
        mp.env_update(handle, side, _dev(E, f64), _dev(bra, f64), _dev(W, f64), _dev(ket, f64), out, prec=prec)
        torch.cuda.synchronize()
        assert_close(out.cpu().numpy(), ref, tol, "left" if side == mp.LEFT else "right")


@pytest.mark.parametrize("prec", [1, 2, 0], ids=["fp32", "bf16x3", "fp64"])
def test_env_update_d256_w271_sampled(mp, handle, prec):
    """The environment update at the full size of the long-range workload (D = 256, d = 2,
    w = 271, both sides; FP32 on the 128 x 128 three-product tiles, split-BF16x3 on 128 x 64): 48
    sampled outputs, each computed by the oracle from the definition restricted to that output
    index (the oracle cannot afford all 17.8 M)."""
    D, d, w = 256, 2, 271
    _say("env_update full size D=256 w=271 sampled", ["fp64", "fp32", "bf16x3"][prec])
    if prec == mp.FP32:  # E . ket and the W contraction (batch D)
        assert handle.product_plan(prec, D * w, d * D, D, 1)["tile"] == (128, 128)
        assert handle.product_plan(prec, d * w, D, d * w, D)["tile"] == (128, 128)
    rng = np.random.default_rng(2562)
    bra, ket, W = _cn(rng, D, d, D), _cn(rng, D, d, D), _cn(rng, w, d, d, w)
    E = _cn(rng, D, w, D)
    f64 = prec == mp.FP64
    tol = {0: 1e-12, 1: 2e-5, 2: 2e-4}[prec]
    idx = [(int(rng.integers(D)), int(rng.integers(w)), int(rng.integers(D))) for _ in range(48)]
    idx += [(0, 0, 0), (D - 1, w - 1, D - 1)]
    out = torch.zeros((D, w, D), dtype=torch.complex128 if f64 else torch.complex64, device="cuda")
    dE, dbra, dW, dket = _dev(E, f64), _dev(bra, f64), _dev(W, f64), _dev(ket, f64)
    for side in (mp.LEFT, mp.RIGHT):
        mp.env_update(handle, side, dE, dbra, dW, dket, out, prec=prec)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        # a reference scale for the element-wise bound: every output entry is a sum of
        # D^2 d^2 w terms of unit variance, so |entry| ~ D d sqrt(w)
        gs, rs = [], []
        for (x, y, z) in idx:
            if side == mp.LEFT:  # E_out[b', beta, b]: restrict bra to b', W to beta, ket to b
                r = ofit.env_left(E, bra[:, :, [x]], W[:, :, :, [y]], ket[:, :, [z]])[0, 0, 0]
            else:                # E_out[a', alpha, a]: restrict bra to a', W to alpha, ket to a
                r = ofit.env_right(E, bra[[x]], W[[y]], ket[[z]])[0, 0, 0]
            gs.append(got[x, y, z])
            rs.append(r)
        gs, rs = np.array(gs), np.array(rs)
        scale = D * d * np.sqrt(w)
        err = float(np.abs(gs - rs).max()) / scale
        print(f"  side {side}: max sampled error {err:.3e} of D d sqrt(w); largest sample "
              f"{np.abs(rs).max() / scale:.2f}", flush=True)
        assert err <= tol, (side, err)


LA_CASES = [  # Dbra_l, Dket_l, Dket_m, Dket_r, Dbra_r, d, w_l, w_m, w_r
    (1, 1, 2, 4, 4, 2, 3, 3, 3),
    (33, 40, 47, 29, 35, 2, 3, 3, 3),
    (64, 64, 64, 64, 64, 2, 6, 6, 6),
    (20, 31, 27, 18, 22, 3, 4, 5, 4),
    (10, 12, 14, 11, 9, 2, 271, 271, 271),
]


@pytest.mark.parametrize("prec64", [True, False], ids=["fp64", "fp32"])
@pytest.mark.parametrize("dims", LA_CASES, ids=[str(c) for c in LA_CASES])
def test_local_apply_parity(mp, handle, dims, prec64):
    Dbl, Dkl, Dkm, Dkr, Dbr, d, wl_, wm, wr = dims
    rng = np.random.default_rng(7 + sum(dims))
    _say("local_apply", "fp64" if prec64 else "fp32", dims)
    L = _cn(rng, Dbl, wl_, Dkl)
    M1, M2 = _cn(rng, Dkl, d, Dkm), _cn(rng, Dkm, d, Dkr)
    W1, W2 = _cn(rng, wl_, d, d, wm), _cn(rng, wm, d, d, wr)
    R = _cn(rng, Dbr, wr, Dkr)
    ref = ofit.theta_two_site(L, M1, W1, M2, W2, R).reshape(Dbl * d, d * Dbr)
    th = torch.zeros((Dbl * d, d * Dbr), dtype=torch.complex128, device="cuda")
    mp.local_apply(handle, _dev(L, prec64), _dev(W1, prec64), _dev(W2, prec64), _dev(M1, prec64),
                   _dev(M2, prec64), _dev(R, prec64), th)
    torch.cuda.synchronize()
    assert_close(th.cpu().numpy(), ref, 1e-12 if prec64 else 2e-5, "theta")


LA1_CASES = [  # Dbra_l, Dket_l, Dket_r, Dbra_r, d, w_l, w_r
    (1, 1, 2, 2, 2, 3, 3),
    (33, 40, 29, 35, 2, 3, 3),
    (64, 64, 64, 64, 2, 6, 6),
    (20, 31, 18, 22, 3, 4, 5),
    (10, 12, 11, 9, 2, 271, 271),
    (128, 128, 128, 128, 2, 271, 271),
]


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("dims", LA1_CASES, ids=[str(c) for c in LA1_CASES])
def test_local_apply_one_site_parity(mp, handle, dims, prec):
    """The one-site projected tensor L M W R (the optimal site at fixed bonds) through local_apply
    with nsites = 1, element-wise against the oracle's definition."""
    Dbl, Dkl, Dkr, Dbr, d, wl_, wr = dims
    rng = np.random.default_rng(11 + sum(dims))
    _say("local_apply one-site", ["fp64", "fp32", "bf16x3"][prec], dims)
    L, M, W, R = _cn(rng, Dbl, wl_, Dkl), _cn(rng, Dkl, d, Dkr), _cn(rng, wl_, d, d, wr), _cn(rng, Dbr, wr, Dkr)
    ref = ofit.local_one_site(L, M, W, R).reshape(Dbl * d, Dbr)
    th = torch.zeros((Dbl * d, Dbr), dtype=torch.complex128, device="cuda")
    f64 = prec == mp.FP64
    mp.local_apply_one_site(handle, _dev(L, f64), _dev(W, f64), _dev(M, f64), _dev(R, f64), th, prec=prec)
    torch.cuda.synchronize()
    assert_close(th.cpu().numpy(), ref, {0: 1e-12, 1: 2e-5, 2: 2e-4}[prec], "theta")


def test_local_apply_rejects_bad_nsites(mp, handle):
    _say("local_apply nsites argument")
    import ctypes
    t = torch.zeros(8, dtype=torch.complex128, device="cuda")
    lib = mp.load()
    arr = (ctypes.c_int * 9)(*([2] * 9))
    rc = lib.local_apply(handle.ptr, 3, mp.FP64, ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                         ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                         ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(t.data_ptr()), arr, None, 0, None)
    assert rc == mp.EINVAL


TR_CASES = [(1, 1), (2, 2), (2, 7), (9, 3), (32, 32), (64, 40), (40, 64), (130, 127), (256, 256), (300, 200),
            (384, 384), (512, 512)]


def _graded(rng, m, n, decay):
    """Random matrix with singular values decaying like exp(-decay * i)."""
    r = min(m, n)
    U, _ = np.linalg.qr(_cn(rng, m, r))
    V, _ = np.linalg.qr(_cn(rng, n, r))
    s = np.exp(-decay * np.arange(r))
    return (U * s) @ V.conj().T


@pytest.mark.parametrize("direction", [0, 1], ids=["left", "right"])
@pytest.mark.parametrize("shape", TR_CASES, ids=[str(c) for c in TR_CASES])
def test_truncate_parity(mp, handle, shape, direction):
    m, n = shape
    rng = np.random.default_rng(m * 1000 + n)
    _say("truncate", shape, "dir", direction)
    X = _cn(rng, m, n) if (m * n) % 2 == 0 else _graded(rng, m, n, 0.3)
    _check_truncate(mp, handle, X, max(1, min(m, n) - 3), direction)


# square matrices take the pivoted-QR preconditioned path: spectra over many decades (graded),
# and exactly rank-deficient ones (the factorisation stops at the zero remainder)
GRADED_SQ = [(64, 0.5, None), (256, 0.12, None), (512, 0.06, None), (200, 0.0, 120), (512, 0.0, 300)]


@pytest.mark.parametrize("direction", [0, 1], ids=["left", "right"])
@pytest.mark.parametrize("case", GRADED_SQ, ids=[str(c) for c in GRADED_SQ])
def test_truncate_square_graded_and_deficient(mp, handle, case, direction):
    n, decay, rank = case
    rng = np.random.default_rng(n + 17 * (rank or 0))
    _say("truncate square", case, "dir", direction)
    if rank is None:
        X = _graded(rng, n, n, decay)
    else:
        X = _cn(rng, n, rank) @ _cn(rng, rank, n)
    _check_truncate(mp, handle, X, n // 2, direction)


# rectangular matrices up to 512 take the pivoted QR too, in either orientation (X = Theta^dag for
# direction 0, Theta for 1, so each shape below gives a tall X in one direction and a wide X, whose
# factorisation stops after min(m, n) steps, in the other): graded spectra and exact rank deficiency
GRADED_RECT = [(96, 320, 0.2, None), (320, 96, 0.2, None), (500, 130, 0.05, None),
               (130, 500, 0.0, 40), (300, 180, 0.0, 60)]


@pytest.mark.parametrize("direction", [0, 1], ids=["left", "right"])
@pytest.mark.parametrize("case", GRADED_RECT, ids=[str(c) for c in GRADED_RECT])
def test_truncate_rect_graded_and_deficient(mp, handle, case, direction):
    m, n, decay, rank = case
    rng = np.random.default_rng(m + 3 * n + 17 * (rank or 0))
    _say("truncate rectangular", case, "dir", direction)
    if rank is None:
        X = _graded(rng, m, n, decay)
    else:
        X = _cn(rng, m, rank) @ _cn(rng, rank, n)
    _check_truncate(mp, handle, X, min(m, n) // 2, direction)


def _check_truncate(mp, handle, X, Dmax, direction):
    m, n = X.shape
    kcap = min(Dmax, m, n)
    A = torch.zeros((m, kcap), dtype=torch.complex128, device="cuda")
    B = torch.zeros((kcap, n), dtype=torch.complex128, device="cuda")
    k = torch.zeros(1, dtype=torch.int32, device="cuda")
    disc = torch.zeros(1, dtype=torch.float64, device="cuda")
    nrm = torch.zeros(1, dtype=torch.float64, device="cuda")
    sig = torch.zeros(min(m, n), dtype=torch.float64, device="cuda")
    mp.truncate(handle, _dev(X), Dmax, 1e-14, direction, A, B, k, disc, nrm, sig)
    torch.cuda.synchronize()
    handle.check_solver()
    U, S, Vh = np.linalg.svd(X, full_matrices=False)
    kk = int(k.item())
    floor = 8 * np.finfo(float).eps * np.sqrt(max(m, n)) * np.linalg.norm(X)
    kref = max(1, min(Dmax, int(np.count_nonzero(S > max(1e-14 * S[0], floor)))))
    assert kk == kref
    assert np.max(np.abs(sig.cpu().numpy() - S)) < 1e-12 * S[0]
    a, b = A.cpu().numpy(), B.cpu().numpy()
    assert not np.any(a[:, kk:]) and not np.any(b[kk:])
    approx = U[:, :kk] @ np.diag(S[:kk]) @ Vh[:kk]
    assert np.max(np.abs(a @ b - approx)) < 1e-11 * S[0]
    iso = a[:, :kk] if direction == 0 else b[:kk].conj().T
    assert np.max(np.abs(iso.conj().T @ iso - np.eye(kk))) < 1e-12
    tot = np.sum(S ** 2)
    assert abs(disc.item() - np.sum(S[kk:] ** 2) / tot) < 1e-12
    assert abs(nrm.item() - np.sqrt(np.sum(S[:kk] ** 2))) < 1e-12 * S[0]


def test_truncate_rank_deficient(mp, handle):
    _say("truncate rank-deficient 64x48 rank 5")
    rng = np.random.default_rng(5)
    X = _cn(rng, 64, 5) @ _cn(rng, 5, 48)
    A = torch.zeros((64, 48), dtype=torch.complex128, device="cuda")
    B = torch.zeros((48, 48), dtype=torch.complex128, device="cuda")
    k = torch.zeros(1, dtype=torch.int32, device="cuda")
    mp.truncate(handle, _dev(X), 64, 1e-12, 0, A, B, k)
    torch.cuda.synchronize()
    assert int(k.item()) == 5
    assert np.max(np.abs(A.cpu().numpy() @ B.cpu().numpy() - X)) < 1e-12 * np.linalg.norm(X, 2)


def _normalise(ms):
    n = ofit.norm(ms)
    out = [m.copy() for m in ms]
    out[0] = out[0] / n
    return out


def _gpu_step(mp, handle, psi, W, D, prec, nsweeps=2, canonical=False):
    dm = mp.DeviceMPS(psi, Dmax=D)
    dw = mp.DeviceMPO([W] * len(psi))
    st = mp.step(handle, dm, dw, nsweeps=nsweeps, prec=prec, input_right_canonical=canonical)
    return dm.to_numpy(), st


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", [(6, 4, 2, 8), (9, 6, 3, 16), (12, 8, 2, 24), (8, 4, 1, 16)], ids=str)
def test_step_parity_random_state(mp, handle, case, prec):
    L, D0, N, D = case
    _say("step random", case, "fp64" if prec == 0 else "fp32")
    rng = np.random.default_rng(L * 7 + D)
    psi = _normalise(wl.random_mps(rng, L, 2, D0))
    W, Wo = mpo_pair(mp, wl.tfim(1.0), N, -0.1j)
    ref, rst = ofit.fit_step(psi, Wo, Dmax=D, nsweeps=2)
    out, st = _gpu_step(mp, handle, psi, W, D, prec)
    infid = 1 - abs(ofit.overlap(out, ref)) ** 2
    assert infid < (1e-12 if prec == 0 else 1e-9), infid
    assert abs(st.norm - rst["norm"]) < (1e-10 if prec == 0 else 1e-6) * rst["norm"]
    assert abs(ofit.norm(out) - 1) < 1e-12
    assert st.visits == 4 * (L - 1)
    assert abs(st.discarded_max - max(rst["discarded"])) < (1e-12 if prec == 0 else 1e-8)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_config1_trajectory(mp, handle, prec):
    """Tiny TFIM configuration (L = 10, g = 1, order 2, dt = 0.05, all-up, D <= 16, 20 steps):
    per-step fidelity against the oracle step from the same input, and the whole trajectory
    against the oracle trajectory and the exact exp(-i t H)."""
    _say("config1 trajectory", "fp64" if prec == 0 else "fp32")
    L, D, dt = 10, 16, 0.05
    H = wl.tfim(1.0)
    W, Wo = mpo_pair(mp, H, 2, -1j * dt)
    psi_gpu = wl.all_up(L)
    psi_or = wl.all_up(L)
    Hd = dense.dense_hamiltonian(ompo.hamiltonian_mpo(H), L)
    v0 = dense.mps_to_dense(wl.all_up(L))
    for step in range(20):
        ref_same, _ = ofit.fit_step(psi_gpu, Wo, Dmax=D, nsweeps=2)
        out, st = _gpu_step(mp, handle, psi_gpu, W, D, prec, canonical=step > 0)
        print(f"  step {step}: bonds {max(st.max_bond, 1)} sweeps {st.svd_sweeps_max}", flush=True)
        delta = 1 - abs(ofit.overlap(out, ref_same)) ** 2
        assert delta < (1e-12 if prec == 0 else 1e-9), (step, delta)
        psi_gpu = out
        psi_or, _ = ofit.fit_step(psi_or, Wo, Dmax=D, nsweeps=2)
    assert 1 - abs(ofit.overlap(psi_gpu, psi_or)) ** 2 < (1e-11 if prec == 0 else 1e-8)
    exact = dense.expm_hermitian(-1j * dt * 20, Hd) @ v0
    assert 1 - abs(np.vdot(dense.mps_to_dense(psi_gpu), exact)) ** 2 < 1e-5


def test_step_rejects_bad_arguments(mp, handle):
    _say("step argument errors")
    psi = wl.all_up(4)
    H = wl.tfim(1.0)
    W, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, 2, -0.1j, mp.V2_EXTENDED)
    dm = mp.DeviceMPS(psi, Dmax=4)
    dw = mp.DeviceMPO([W] * 4)
    with pytest.raises(mp.MpoevoError) as e:
        mp.step(handle, dm, dw, nsweeps=0)
    assert e.value.code == mp.EINVAL
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(mp.MpoevoError) as e:
        mp.step(handle, dm, dw, workspace=ws)
    assert e.value.code == mp.ENOMEM


def test_step_profile_mode_matches_plain_step(mp, handle):
    """The event-timed step computes the same state and reports positive kernel-class times."""
    _say("step profile mode L=8 D=8")
    rng = np.random.default_rng(3)
    psi = _normalise(wl.random_mps(rng, 8, 2, 4))
    H = wl.tfim(1.0)
    W, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, 2, -0.1j, mp.V2_EXTENDED)
    a, sa = _gpu_step(mp, handle, psi, W, 8, 0)
    dm = mp.DeviceMPS(psi, Dmax=8)
    sb = mp.step(handle, dm, mp.DeviceMPO([W] * 8), prec=0, profile=True)
    b = dm.to_numpy()
    assert 1 - abs(ofit.overlap(a, b)) ** 2 < 1e-13
    p = sb.profile
    assert p["n_jacobi"] == sa.visits and p["t_jacobi_ms"] > 0 and p["jacobi_gflop"] > 0
    assert p["n_gemm"] > 0 and p["t_gemm_ms"] > 0 and p["gemm_gflop"] > 0
    assert p["n_wmix"] > 0 and p["wmix_gbyte"] > 0


def test_step_warm_started_truncations_match_cold_and_oracle(mp, handle):
    """Preconditioned Jacobi (the unitary the previous truncation of a bond left behind) gives the
    same trajectory as cold starts and as the oracle, with fewer sweeps once the bases exist."""
    _say("step warm start L=12 D=8 saturated random state, 4 steps")
    L, D = 12, 8  # bonds 3..7 have square 16 x 16 bond matrices
    rng = np.random.default_rng(11)
    psi = _normalise(wl.random_mps(rng, L, 2, D))
    H = wl.tfim(1.5)
    W, Wo = mpo_pair(mp, H, 2, -0.1j)
    dw = mp.DeviceMPO([W] * L)
    warm = mp.DeviceMPS(psi, Dmax=D)
    cold = mp.DeviceMPS(psi, Dmax=D)
    ws_w = mp.step_workspace(warm, dw, mp.FP64)
    ws_c = torch.empty_like(ws_w)
    ref = psi
    tot_w, tot_c = [], []
    for s in range(4):
        sw = mp.step(handle, warm, dw, prec=mp.FP64, input_right_canonical=s > 0, workspace=ws_w)
        sc = mp.step(handle, cold, dw, prec=mp.FP64, input_right_canonical=s > 0, workspace=ws_c,
                     svd_cold_start=True)
        ref, _ = ofit.fit_step(ref, Wo, Dmax=D, nsweeps=2)
        a, b = warm.to_numpy(), cold.to_numpy()
        assert 1 - abs(ofit.overlap(a, b)) ** 2 < 1e-12, s
        assert 1 - abs(ofit.overlap(a, ref)) ** 2 < 1e-10, s
        assert abs(sw.norm - sc.norm) < 1e-11 * sc.norm
        tot_w.append(sw.svd_sweeps_total)
        tot_c.append(sc.svd_sweeps_total)
    print("total sweeps per step: warm", tot_w, "cold", tot_c, flush=True)
    assert all(t > 0 for t in tot_w + tot_c)
    assert sum(tot_w[1:]) < sum(tot_c[1:])


def test_fp32_step_sweep_end_keeps_fidelity_and_isometries(mp, handle):
    """FP32 steps end the Jacobi iteration after the sweep whose largest relative inner product is
    below kSvdAcceptFp32 (quadratic convergence leaves about its square). On a saturated state
    (square 128 x 128 bond matrices, warm-started visits), three chained FP32 steps each stay within
    infidelity 1e-10 of the FP64 step from the same input, and the right-canonical sites stay
    isometric to 1e-9."""
    _say("fp32 sweep end L=14 D=64 saturated, 3 steps")
    L, D = 14, 64
    rng = np.random.default_rng(23)
    psi = _normalise(wl.random_mps(rng, L, 2, D))
    H = wl.tfim(1.5)
    W, Wo = mpo_pair(mp, H, 2, -0.1j)
    dw = mp.DeviceMPO([W] * L)
    d32 = mp.DeviceMPS(psi, Dmax=D)
    ws32 = mp.step_workspace(d32, dw, mp.FP32)
    sw32, sw64 = [], []
    for s in range(3):
        before = d32.to_numpy()
        st32 = mp.step(handle, d32, dw, prec=mp.FP32, input_right_canonical=s > 0, workspace=ws32)
        d64 = mp.DeviceMPS(before, Dmax=D)
        st64 = mp.step(handle, d64, dw, prec=mp.FP64, input_right_canonical=s > 0)
        a, b = d32.to_numpy(), d64.to_numpy()
        infid = 1 - abs(ofit.overlap(a, b)) ** 2
        ref, rst = ofit.fit_step(before, Wo, Dmax=D, nsweeps=2)
        infid_or = 1 - abs(ofit.overlap(a, ref)) ** 2
        assert infid_or < 1e-9, (s, infid_or)
        assert abs(st32.norm - rst["norm"]) < 1e-6 * rst["norm"]
        iso = max(float(np.max(np.abs(B.reshape(B.shape[0], -1) @ B.reshape(B.shape[0], -1).conj().T
                                      - np.eye(B.shape[0])))) for B in a[1:])
        print(f"  step {s}: infidelity {infid:.2e} (oracle {infid_or:.2e}) isometry {iso:.1e} sweeps fp32 {st32.svd_sweeps_total}"
              f" fp64 {st64.svd_sweeps_total}", flush=True)
        assert infid < 1e-10, (s, infid)
        assert iso < 1e-9, (s, iso)
        sw32.append(st32.svd_sweeps_total)
        sw64.append(st64.svd_sweeps_total)
    assert all(t > 0 for t in sw32 + sw64)


def _hamiltonian_mpo_from_blocks(H):
    """[[I, C, Dloc], [0, A, B], [0, 0, I]] assembled here from the Jordan blocks (Sec. 2.3)."""
    d, chi = H.Dloc.shape[0], H.B.shape[0]
    w = chi + 2
    W = np.zeros((w, d, d, w), dtype=np.complex128)
    W[0, :, :, 0] = np.eye(d)
    W[w - 1, :, :, w - 1] = np.eye(d)
    W[0, :, :, w - 1] = H.Dloc
    for k in range(chi):
        W[0, :, :, 1 + k] = H.C[k]
        W[1 + k, :, :, w - 1] = H.B[k]
        for l in range(chi):
            W[1 + k, :, :, 1 + l] = H.A[k, l]
    return W


@pytest.mark.parametrize("L,D", [(8, 8), (11, 20)], ids=str)
def test_expectation_energy_local_norm(mp, handle, L, D):
    """<psi|O|psi> on the device (FP64) against the oracle: the TFIM energy through the Hamiltonian
    MPO, <Z_3> through a bond-1 MPO, the norm, and <psi|W|psi> of the evolution MPO."""
    _say("expectation", L, D)
    rng = np.random.default_rng(L + D)
    psi = wl.random_mps(rng, L, 2, D)
    dm = mp.DeviceMPS(psi, Dmax=D)
    H = wl.tfim(1.3)
    Wh = _hamiltonian_mpo_from_blocks(H)
    w = Wh.shape[0]
    e0, e1 = np.zeros(w, complex), np.zeros(w, complex)
    e0[0], e1[w - 1] = 1.0, 1.0
    ref = ofit.mpo_expectation(psi, [Wh] * L, e0, e1)
    got = mp.expectation(handle, dm, mp.DeviceMPO([Wh] * L), left=0, right=w - 1)
    assert abs(got - ref) < 1e-12 * max(1.0, abs(ref)), (got, ref)
    nrm = ofit.overlap(psi, psi)
    Id = np.eye(2, dtype=np.complex128).reshape(1, 2, 2, 1)
    Z3 = [Id] * L
    Z3[3] = wl.SZ.reshape(1, 2, 2, 1)
    got = mp.expectation(handle, dm, mp.DeviceMPO(Z3))
    ref = ofit.expect_local(psi, wl.SZ, 3) * nrm
    assert abs(got - ref) < 1e-12 * abs(nrm)
    got = mp.expectation(handle, dm, mp.DeviceMPO([Id] * L))
    assert abs(got - nrm) < 1e-12 * abs(nrm)
    W, Wo = mpo_pair(mp, H, 2, -0.1j)
    l0 = np.zeros(W.shape[0], complex)
    l0[0] = 1.0
    ref = ofit.mpo_expectation(psi, [Wo] * L, l0, l0)
    got = mp.expectation(handle, dm, mp.DeviceMPO([W] * L))
    assert abs(got - ref) < 1e-12 * abs(nrm)


def test_expectation_rejects_bad_levels(mp, handle):
    _say("expectation argument errors")
    psi = wl.all_up(4)
    dm = mp.DeviceMPS(psi, Dmax=2)
    Wh = _hamiltonian_mpo_from_blocks(wl.tfim(1.0))
    with pytest.raises(mp.MpoevoError) as e:
        mp.expectation(handle, dm, mp.DeviceMPO([Wh] * 4), left=0, right=Wh.shape[0])
    assert e.value.code == mp.EINVAL


def _lr_blocks(g):
    import json, os
    fit = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lr_fit_K6.json")))
    return wl.lr_ising(np.array(fit["coeffs"]), np.array(fit["lambdas"]), g)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_step_parity_long_range_order3(mp, handle, prec):
    """Long-range Ising (J(r) = r^-2 as six exponentials, g = 1), order-3 extended MPO (w = 271):
    one step against the oracle from the same random state."""
    _say("step long-range order 3 w=271 L=6 D=8", "fp64" if prec == 0 else "fp32")
    H = _lr_blocks(1.0)
    W, Wo = mpo_pair(mp, H, 3, -0.1j)
    assert W.shape[0] == 271
    rng = np.random.default_rng(31)
    psi = _normalise(wl.random_mps(rng, 6, 2, 4))
    ref, rst = ofit.fit_step(psi, Wo, Dmax=8, nsweeps=2)
    out, st = _gpu_step(mp, handle, psi, W, 8, prec)
    infid = 1 - abs(ofit.overlap(out, ref)) ** 2
    assert infid < (1e-12 if prec == 0 else 1e-9), infid
    assert abs(st.norm - rst["norm"]) < (1e-10 if prec == 0 else 1e-6) * rst["norm"]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_split_composite_step(mp, handle, prec):
    """Splitting composite (Sec. 8.3): the first-order MPO at t2 tau, then at t1 tau, through two
    step calls on the GPU, against the oracle's two fits with its own first-order MPOs (same
    order), and against the exact exp(tau H) psi: the unnormalised result (output times the two
    fitted norms) differs from it by O(dt^3), where one first-order step alone is O(dt^2)."""
    L, D = 8, 16
    _say("split composite L=8 D=16", "fp64" if prec == 0 else "fp32")
    H = wl.tfim(1.0)
    rng = np.random.default_rng(5)
    psi = _normalise(wl.random_mps(rng, L, 2, 4))
    v0 = dense.mps_to_dense(psi)
    Hd = dense.dense_hamiltonian(ompo.hamiltonian_mpo(H), L)
    errs = []
    for dt in (0.1, 0.05):
        tau = -1j * dt
        Wb, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, 1, mp.SPLIT_T2 * tau, mp.V2_EXTENDED)
        Wa, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, 1, mp.SPLIT_T1 * tau, mp.V2_EXTENDED)
        assert Wa.shape[0] == Wb.shape[0] == 2
        dm = mp.DeviceMPS(psi, Dmax=D)
        s1, s2 = mp.split_step(handle, dm, mp.DeviceMPO([Wb] * L), mp.DeviceMPO([Wa] * L), prec=prec)
        out = dm.to_numpy()
        mid, r1 = ofit.fit_step(psi, ompo.build_mpo(H, 1, ompo.SPLIT_T2 * tau, "V2"), Dmax=D)
        ref, r2 = ofit.fit_step(mid, ompo.build_mpo(H, 1, ompo.SPLIT_T1 * tau, "V2"), Dmax=D)
        infid = 1 - abs(ofit.overlap(out, ref)) ** 2
        assert infid < (1e-12 if prec == 0 else 1e-9), (dt, infid)
        tol = 1e-10 if prec == 0 else 1e-6
        assert abs(s1.norm - r1["norm"]) < tol * r1["norm"] and abs(s2.norm - r2["norm"]) < tol * r2["norm"]
        exact = dense.expm_hermitian(tau, Hd) @ v0
        errs.append(np.linalg.norm(dense.mps_to_dense(out) * (s1.norm * s2.norm) - exact))
    slope = np.log(errs[0] / errs[1]) / np.log(2)
    assert slope > 3 - 0.2, (errs, slope)


def _tfim_h_mpo(H):
    """Hamiltonian MPO over levels (1, 2, 3) of a chi = 1 chain, written out (product-side input)."""
    Hm = np.zeros((3, 2, 2, 3), dtype=np.complex128)
    Hm[0, :, :, 0] = Hm[2, :, :, 2] = np.eye(2)
    Hm[0, :, :, 1], Hm[1, :, :, 2], Hm[0, :, :, 2] = H.C[0], H.B[0], H.Dloc
    return Hm


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_thermal_purification(mp, handle, prec):
    """Finite temperature by purification (d = 4 sites: physical and ancilla legs): the order-2
    MPO at tau = -delta on the physical legs, 10 steps from beta = 0 to beta = 1, each against the
    oracle's fit from the same input; the device energy (FP64 expectation of H on the physical
    legs) against the oracle's trajectory and the exact thermal energy of the dense Hamiltonian."""
    L, D, delta, K = 8, 32, 0.05, 10
    _say("thermal purification L=8 d=4 D=32", "fp64" if prec == 0 else "fp32")
    H = wl.tfim(1.0)
    W, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, 2, -delta, mp.V2_EXTENDED)
    Wo = ompo.purify(ompo.build_mpo(H, 2, -delta, "V2"))
    dm = mp.DeviceMPS(wl.infinite_temperature(L), Dmax=D)
    dw = mp.DeviceMPO([mp.purify_mpo(W)] * L)
    traj = wl.infinite_temperature(L)
    for k in range(K):
        same, _ = ofit.fit_step(dm.to_numpy(), Wo, Dmax=D)
        mp.step(handle, dm, dw, prec=prec, input_right_canonical=k > 0)
        infid = 1 - abs(ofit.overlap(dm.to_numpy(), same)) ** 2
        assert infid < (1e-12 if prec == 0 else 1e-9), (k, infid)
        traj, _ = ofit.fit_step(traj, Wo, Dmax=D)
    Hp = mp.purify_mpo(_tfim_h_mpo(H))
    e_gpu = mp.expectation(handle, dm, mp.DeviceMPO([Hp] * L), 0, Hp.shape[0] - 1).real
    Ho = ompo.purify(ompo.hamiltonian_mpo(H))
    w = Ho.shape[0]
    e_or = (ofit.mpo_expectation(traj, [Ho] * L, dense.boundary(w, 0), dense.boundary(w, w - 1))
            / ofit.overlap(traj, traj)).real
    lam = np.linalg.eigvalsh(dense.dense_hamiltonian(ompo.hamiltonian_mpo(H), L))
    p = np.exp(-1.0 * (lam - lam.min()))
    e_ex = float((lam * p).sum() / p.sum())
    assert abs(e_gpu - e_or) < (1e-10 if prec == 0 else 1e-5) * abs(e_ex), (e_gpu, e_or)
    assert abs(e_gpu - e_ex) < 3e-3, (e_gpu, e_ex)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("N", [1, 2, 3])
def test_cylinder_step_parity(mp, handle, N, prec):
    """TFIM on a W = 4 spiral cylinder (12 sites, h = 2): one step of the order-N MPO (bond 5,
    21, 93: register and product paths of the W contraction) against the oracle's fit with its own
    MPO from the same random state."""
    L, D, dt = 12, 16, 0.1
    _say("cylinder W=4 step", N, "fp64" if prec == 0 else "fp32")
    H = wl.tfim_cylinder(4, 2.0)
    psi = _normalise(wl.random_mps(np.random.default_rng(40 + N), L, 2, 6))
    W, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, N, -1j * dt, mp.V2_EXTENDED)
    assert W.shape[0] == {1: 5, 2: 21, 3: 93}[N]
    ref, rst = ofit.fit_step(psi, ompo.build_mpo(H, N, -1j * dt, "V2"), Dmax=D)
    out, st = _gpu_step(mp, handle, psi, W, D, prec)
    infid = 1 - abs(ofit.overlap(out, ref)) ** 2
    assert infid < (1e-12 if prec == 0 else 1e-9), infid
    assert abs(st.norm - rst["norm"]) < (1e-10 if prec == 0 else 1e-6) * rst["norm"]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_xxz_step_conserves_charge(mp, handle, prec):
    """Spin-1/2 XXZ chain (Delta = 0.5), order-2 MPO (bond 13), from the Neel state (5 up spins
    of 10): two steps against the oracle's fits, and the U(1) charge conserved by the device
    path: <sum Sz> = 0 and its variance <(sum Sz)^2> - <sum Sz>^2 = 0 after each step."""
    L, D, dt = 10, 16, 0.1
    _say("xxz step L=10 D=16", "fp64" if prec == 0 else "fp32")
    H = wl.xxz(0.5)
    W, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, 2, -1j * dt, mp.V2_EXTENDED)
    assert W.shape[0] == 13
    Wo = ompo.build_mpo(H, 2, -1j * dt, "V2")
    up, dn = np.array([1, 0], dtype=np.complex128), np.array([0, 1], dtype=np.complex128)
    psi = [(up if i % 2 == 0 else dn).reshape(1, 2, 1) for i in range(L)]
    sz = 0.5 * wl.SZ
    I2 = np.eye(2, dtype=np.complex128)
    S1 = np.zeros((2, 2, 2, 2), dtype=np.complex128)  # sum Sz: [[I, Sz], [0, I]]
    S1[0, :, :, 0] = S1[1, :, :, 1] = I2
    S1[0, :, :, 1] = sz
    S2 = np.zeros((3, 2, 2, 3), dtype=np.complex128)  # (sum Sz)^2: [[I, 2Sz, Sz^2], [0, I, Sz], [0, 0, I]]
    S2[0, :, :, 0] = S2[1, :, :, 1] = S2[2, :, :, 2] = I2
    S2[0, :, :, 1], S2[0, :, :, 2], S2[1, :, :, 2] = 2 * sz, sz @ sz, sz
    dm = mp.DeviceMPS(psi, Dmax=D)
    dw = mp.DeviceMPO([W] * L)
    d1, d2 = mp.DeviceMPO([S1] * L), mp.DeviceMPO([S2] * L)
    ref = psi
    for k in range(2):
        ref, _ = ofit.fit_step(ref, Wo, Dmax=D)
        mp.step(handle, dm, dw, prec=prec, input_right_canonical=k > 0)
        infid = 1 - abs(ofit.overlap(dm.to_numpy(), ref)) ** 2
        assert infid < (1e-12 if prec == 0 else 1e-9), (k, infid)
        m1 = mp.expectation(handle, dm, d1, 0, 1).real
        m2 = mp.expectation(handle, dm, d2, 0, 2).real
        tol = 1e-10 if prec == 0 else 1e-6
        assert abs(m1) < tol and abs(m2 - m1 * m1) < tol, (k, m1, m2)


@pytest.mark.parametrize("prec", [1, 0], ids=["fp32", "fp64"])
def test_step_long_range_order3_d64(mp, handle, prec):
    """The order-3 long-range MPO (w = 271) on L = 14 at D = 64 (middle bonds saturated): the
    products of the step run on the 128 x 64 tile (E ket: 17344 x 128 outputs). One step against
    the oracle's fit (its own MPO) from the same random state."""
    L, D = 14, 64
    _say("step long-range order 3 w=271 L=14 D=64", "fp64" if prec == 0 else "fp32")
    plan = handle.product_plan(prec, D * 271, 2 * D, D)
    print("  plan of the E ket product:", plan, flush=True)
    if prec == mp.FP32:
        assert plan["tile"] == (128, 64)
    H = _lr_blocks(1.0)
    W, Wo = mpo_pair(mp, H, 3, -0.1j)
    psi = _normalise(wl.random_mps(np.random.default_rng(1464), L, 2, D))
    ref, rst = ofit.fit_step(psi, Wo, Dmax=D, nsweeps=2)
    out, st = _gpu_step(mp, handle, psi, W, D, prec)
    infid = 1 - abs(ofit.overlap(out, ref)) ** 2
    print(f"  infidelity {infid:.3e}, norm {st.norm:.12f} vs {rst['norm']:.12f}", flush=True)
    assert infid < (1e-12 if prec == 0 else 1e-9), infid
    assert abs(st.norm - rst["norm"]) < (1e-10 if prec == 0 else 1e-6) * rst["norm"]
    assert abs(st.discarded_sum - sum(rst["discarded"])) < (1e-11 if prec == 0 else 1e-7)


def test_default_workspace_survives_other_allocations(mp, handle):
    """step() without a workspace keeps one per MPS object: the truncation preconditioners it
    leaves there survive other allocations made between two steps (which would otherwise reuse a
    freed temporary and overwrite them), so two such steps match the oracle's two fits."""
    L, D = 12, 8
    _say("default workspace L=12 D=8, scribbled allocations between two steps")
    psi = _normalise(wl.random_mps(np.random.default_rng(77), L, 2, D))
    W, Wo = mpo_pair(mp, wl.tfim(1.5), 2, -0.1j)
    dm = mp.DeviceMPS(psi, Dmax=D)
    dw = mp.DeviceMPO([W] * L)
    mp.step(handle, dm, dw, prec=mp.FP64)
    nbytes = mp.step_workspace(dm, dw, mp.FP64).numel()
    junk = [torch.full((nbytes,), 0x5a, dtype=torch.uint8, device="cuda") for _ in range(3)]
    torch.cuda.synchronize()
    st = mp.step(handle, dm, dw, prec=mp.FP64, input_right_canonical=True)
    del junk
    ref, _ = ofit.fit_step(psi, Wo, Dmax=D)
    ref, rst = ofit.fit_step(ref, Wo, Dmax=D)
    infid = 1 - abs(ofit.overlap(dm.to_numpy(), ref)) ** 2
    assert infid < 1e-12, infid
    assert abs(st.norm - rst["norm"]) < 1e-10 * rst["norm"]


def test_tile_tuner(mp, handle):
    """The tile tuner: with tuning on, the first environment update of a shape times the
    candidate plans and keeps one (the plan query then reports it as tuned); the tuned product
    still matches the oracle element-wise; frozen mode keeps the table; clearing restores the
    fixed rule."""
    dims = (200, 200, 200, 200, 2, 6, 6)
    _say("tile tuner", dims)
    Dbl, Dkl, Dbr, Dkr, d, wl_, wr = dims
    rng = np.random.default_rng(5151)
    bra, ket, W = _cn(rng, Dbl, d, Dbr), _cn(rng, Dkl, d, Dkr), _cn(rng, wl_, d, d, wr)
    E = _cn(rng, Dbl, wl_, Dkl)
    ref = ofit.env_left(E, bra, W, ket)
    shape = (Dbl * wl_, d * Dkr, Dkl)  # the E ket product
    try:
        assert not handle.product_plan(mp.FP32, *shape)["tuned"]
        handle.set_tuning(mp.TUNE_ON, clear=True)
        for _ in range(2):
            out = torch.zeros(ref.shape, dtype=torch.complex64, device="cuda")
            mp.env_update(handle, mp.LEFT, _dev(E, False), _dev(bra, False), _dev(W, False), _dev(ket, False), out)
            torch.cuda.synchronize()
            assert_close(out.cpu().numpy(), ref, 2e-5, "tuned env_update")
        plan = handle.product_plan(mp.FP32, *shape)
        print("  tuned plan", plan, flush=True)
        assert plan["tuned"] and plan["entries"] >= 2
        handle.set_tuning(mp.TUNE_FROZEN)
        assert handle.product_plan(mp.FP32, *shape)["tuned"]
        handle.set_tuning(mp.TUNE_OFF, clear=True)
        p = handle.product_plan(mp.FP32, *shape)
        assert not p["tuned"] and p["entries"] == 0
    finally:
        handle.set_tuning(mp.TUNE_OFF, clear=True)


ONE_SITE_CASES = [(8, 8, 2), (12, 16, 2), (10, 32, 3), (9, 256, 1),
                  (18, 256, 2)]  # L, Dmax (bonds at their cap), order; the last at the full QR width (512 x 256)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", ONE_SITE_CASES, ids=str)
def test_one_site_step_parity(mp, handle, case, prec):
    """One-site updates at fixed bonds (FP64 Householder QR of each projected site tensor) against
    the oracle's one-site fit from the same state: gauge-invariant overlap and the fitted norm."""
    L, D, N = case
    _say("one-site step", case, "fp64" if prec == 0 else "fp32")
    psi = _normalise(wl.random_mps(np.random.default_rng(300 + L + D), L, 2, D))
    W, Wo = mpo_pair(mp, wl.tfim(1.2), N, -0.1j)
    ref, rst = ofit.fit_step_one_site(psi, Wo, nsweeps=2)
    dm = mp.DeviceMPS(psi, Dmax=D)
    st = mp.step(handle, dm, mp.DeviceMPO([W] * L), prec=prec, nsites=1)
    out = dm.to_numpy()
    infid = 1 - abs(ofit.overlap(out, ref)) ** 2
    print(f"  infidelity {infid:.3e} norm {st.norm:.14f} vs {rst['norm']:.14f}", flush=True)
    assert [m.shape for m in out] == [m.shape for m in ref]
    assert infid < (1e-12 if prec == 0 else 1e-9), infid
    assert abs(st.norm - rst["norm"]) < (1e-10 if prec == 0 else 1e-6) * rst["norm"]
    assert abs(ofit.norm(out) - 1) < 1e-12
    assert st.visits == 4 * (L - 1) + 1 and st.discarded_sum == 0.0 and st.svd_sweeps_max == 0


@pytest.mark.parametrize("prec", [1, 0], ids=["fp32", "fp64"])
def test_one_site_step_long_range_d64(mp, handle, prec):
    """One-site updates with the order-3 long-range MPO (w = 271) at L = 14, D = 64."""
    L, D = 14, 64
    _say("one-site step long-range w=271 L=14 D=64", "fp64" if prec == 0 else "fp32")
    W, Wo = mpo_pair(mp, _lr_blocks(1.0), 3, -0.1j)
    psi = _normalise(wl.random_mps(np.random.default_rng(1465), L, 2, D))
    ref, rst = ofit.fit_step_one_site(psi, Wo, nsweeps=2)
    dm = mp.DeviceMPS(psi, Dmax=D)
    st = mp.step(handle, dm, mp.DeviceMPO([W] * L), prec=prec, nsites=1, profile=True)
    infid = 1 - abs(ofit.overlap(dm.to_numpy(), ref)) ** 2
    print(f"  infidelity {infid:.3e}; kernels: " +
          ", ".join(f"{k['kind']} {k['ms']:.2f} ms" for k in st.profile["kernels"][:4]), flush=True)
    assert infid < (1e-12 if prec == 0 else 1e-9), infid
    assert abs(st.norm - rst["norm"]) < (1e-10 if prec == 0 else 1e-6) * rst["norm"]
    assert any(k["kind"] == "householder_qr" for k in st.profile["kernels"])


def test_auto_update_picks_by_bond_saturation(mp, handle):
    """nsites = -1: one-site updates when every bond is at its largest value, else two-site."""
    L, D = 10, 16
    _say("automatic one-/two-site choice L=10 D=16")
    W, Wo = mpo_pair(mp, wl.tfim(0.8), 2, -0.1j)
    dw = mp.DeviceMPO([W] * L)
    full = _normalise(wl.random_mps(np.random.default_rng(21), L, 2, D))  # bonds at the cap
    part = _normalise(wl.random_mps(np.random.default_rng(22), L, 2, 6))  # bonds below it
    for psi, fit in ((full, ofit.fit_step_one_site), (part, lambda p, W_: ofit.fit_step(p, W_, Dmax=D))):
        ref, _ = fit(psi, Wo)
        dm = mp.DeviceMPS(psi, Dmax=D)
        st = mp.step(handle, dm, dw, prec=mp.FP64, nsites=mp.NSITES_AUTO)
        assert 1 - abs(ofit.overlap(dm.to_numpy(), ref)) ** 2 < 1e-12
        assert st.visits == (4 * (L - 1) + 1 if fit is ofit.fit_step_one_site else 4 * (L - 1))


def test_one_site_rejects_unsupported_shapes(mp, handle):
    _say("one-site shape errors")
    L = 6
    W, _ = mpo_pair(mp, wl.tfim(1.0), 2, -0.1j)
    dm = mp.DeviceMPS(wl.all_up(L), Dmax=512)  # d Dmax = 1024 > 512
    with pytest.raises(mp.MpoevoError) as e:
        mp.step(handle, dm, mp.DeviceMPO([W] * L), nsites=1)
    assert e.value.code == mp.ESHAPE
    with pytest.raises(mp.MpoevoError) as e:
        mp.step(handle, dm, mp.DeviceMPO([W] * L), nsites=3)
    assert e.value.code == mp.EINVAL


@pytest.mark.parametrize("L,Db,Dk", [(7, 4, 9), (10, 16, 6)], ids=str)
def test_overlap_fp64(mp, handle, L, Db, Dk):
    """<bra| W |ket> on the device in FP64 against the oracle, bra and ket with different bonds."""
    _say("overlap", L, Db, Dk)
    rng = np.random.default_rng(L * 31 + Db)
    bra, ket = wl.random_mps(rng, L, 2, Db), wl.random_mps(rng, L, 2, Dk)
    W, Wo = mpo_pair(mp, wl.tfim(1.1), 2, -0.2j)
    e0 = np.zeros(W.shape[0], complex)
    e0[0] = 1.0
    ref = ofit.mpo_overlap(bra, [Wo] * L, ket, e0, e0)
    got = mp.overlap(handle, mp.DeviceMPS(bra, Dmax=Db), mp.DeviceMPO([W] * L), mp.DeviceMPS(ket, Dmax=Dk))
    assert abs(got - ref) < 1e-12 * abs(ref), (got, ref)
