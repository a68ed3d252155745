"""Helpers shared by the GPU parity tests (imported by them; no tests here).

Tolerance checks are element-wise against the largest oracle entry, so that a single wrong
output cannot hide in a norm: max |gpu - oracle| <= tol * max |oracle|, and also the relative
Frobenius error <= tol.

Every time-evolution MPO handed to the oracle comes from the oracle's own construction
(oracle.mpo.build_mpo); the library's mpo_build supplies only the device side.
"""
import numpy as np

from oracle import mpo as ompo


def say(*a):
    print("[case]", *a, flush=True)


def assert_close(got, ref, tol, what=""):
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    scale = max(float(np.abs(ref).max()), 1e-300)
    elem = float(np.abs(got - ref).max()) / scale
    fro = float(np.linalg.norm((got - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))
    print(f"  {what} element-wise {elem:.3e} (of max |ref|), Frobenius {fro:.3e}", flush=True)
    assert elem <= tol and fro <= tol, (what, elem, fro, tol)
    return elem, fro


def mpo_pair(mp, H, N, tau, variant="V2"):
    """(W for the device from the library's builder, W for the oracle from the oracle's)."""
    W_lib, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, N, tau,
                            mp.V2_EXTENDED if variant == "V2" else mp.V1_EXACT)
    W_or = ompo.build_mpo(H, N, tau, variant)
    assert W_lib.shape == W_or.shape
    return W_lib, W_or


def normalise(ms, norm_fn):
    n = norm_fn(ms)
    out = [m.copy() for m in ms]
    out[0] = out[0] / n
    return out
