"""Host-side checks of the C ABI library (no GPU needed): it loads, exports every symbol the
header declares, and its host `mpo_build` agrees with the oracle's construction."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import mpo as omp
from paper_2302_14181_amd import mpoevo
from paper_2302_14181_amd import workloads as wl

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "mpoevo.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_library_loads_and_exports_header_symbols():
    lib = mpoevo.load()
    declared = _declared_functions()
    assert set(declared) == set(mpoevo.exported_symbols())
    for name in declared:
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.mpoevo_version()


@pytest.mark.parametrize("variant,vname", [(mpoevo.V1_EXACT, "V1"), (mpoevo.V2_EXTENDED, "V2")])
@pytest.mark.parametrize("chi,N", [(1, 1), (1, 2), (1, 3), (1, 4), (2, 2), (2, 3), (3, 2), (2, 4)])
def test_mpo_build_matches_oracle(chi, N, variant, vname):
    H = wl.random_blocks(np.random.default_rng(100 * chi + N), 2, chi)
    tau = 0.13 - 0.27j
    W, _ = mpoevo.mpo_build(H.A, H.B, H.C, H.Dloc, N, tau, variant)
    ref = omp.build_mpo(H, N, tau, vname)
    assert W.shape == ref.shape
    assert np.max(np.abs(W - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref)))


def test_mpo_build_level_charges_match_oracle():
    H = wl.xxz(0.5)
    for N in (1, 2, 3):
        W, q = mpoevo.mpo_build(H.A, H.B, H.C, H.Dloc, N, -0.1j, mpoevo.V2_EXTENDED,
                                H.inner_charge, H.phys_charge)
        assert np.array_equal(q, omp.level_charges(H, N, -0.1j, "V2"))


def test_mpo_build_d3_matches_oracle():
    H = wl.random_blocks(np.random.default_rng(9), 3, 2)
    W, _ = mpoevo.mpo_build(H.A, H.B, H.C, H.Dloc, 3, 0.2 + 0.1j, mpoevo.V2_EXTENDED)
    ref = omp.build_mpo(H, 3, 0.2 + 0.1j, "V2")
    assert np.max(np.abs(W - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref)))


def test_mpo_build_errors():
    lib = mpoevo.load()
    H = wl.tfim(1.0)
    with pytest.raises(mpoevo.MpoevoError) as e:
        mpoevo.mpo_build(H.A, H.B, H.C, H.Dloc, 5, 0.1)
    assert e.value.code == mpoevo.EINVAL
    with pytest.raises(mpoevo.MpoevoError) as e:
        mpoevo.mpo_build(H.A, H.B, H.C, H.Dloc, 2, complex(np.nan, 0))
    assert e.value.code == mpoevo.ENONFINITE
    bad = H.Dloc.copy()
    bad[0, 0] = np.inf
    with pytest.raises(mpoevo.MpoevoError) as e:
        mpoevo.mpo_build(H.A, H.B, H.C, bad, 2, 0.1)
    assert e.value.code == mpoevo.ENONFINITE
    with pytest.raises(mpoevo.MpoevoError) as e:
        mpoevo.mpo_build(H.A, H.B, H.C, H.Dloc, 2, 0.1, variant=7)
    assert e.value.code == mpoevo.EINVAL
    # capacity too small
    w = ctypes.c_int(0)
    A = np.ascontiguousarray(H.A); B = np.ascontiguousarray(H.B); C = np.ascontiguousarray(H.C)
    D = np.ascontiguousarray(H.Dloc)
    out = np.zeros(4, dtype=np.complex128)
    rc = lib.mpo_build(2, 1, mpoevo._dptr(A.view(np.float64)), mpoevo._dptr(B.view(np.float64)),
                       mpoevo._dptr(C.view(np.float64)), mpoevo._dptr(D.view(np.float64)), 2, 0.1, 0.0,
                       1, None, None, ctypes.byref(w), mpoevo._dptr(out.view(np.float64)), 4, None)
    assert rc == mpoevo.ENOMEM and w.value == 3
    assert b"capacity" in lib.mpoevo_last_error(None)


def test_workspace_queries():
    assert mpoevo.workspace_size(mpoevo.CALL_TRUNCATE, [512, 512], mpoevo.FP64) > 512 * 512 * 16
    # up to 512 the truncation goes through the pivoted QR: besides the 32 MiB product scratch its
    # workspace holds X, R^dag and two candidate columns per workgroup (at least 4 x 512^2 complex)
    for m, n in [(512, 512), (256, 512), (512, 130)]:
        need = (32 << 20) + 4 * max(m, n) * min(m, n) * 16
        assert mpoevo.workspace_size(mpoevo.CALL_TRUNCATE, [m, n], mpoevo.FP64) >= need, (m, n)
    s64 = mpoevo.workspace_size(mpoevo.CALL_STEP, [16, 2, 32, 3], mpoevo.FP64)
    s32 = mpoevo.workspace_size(mpoevo.CALL_STEP, [16, 2, 32, 3], mpoevo.FP32)
    assert s64 > 0 and s32 > 0
    with pytest.raises(mpoevo.MpoevoError) as e:
        mpoevo.workspace_size(mpoevo.CALL_STEP, [1, 2, 32, 3], mpoevo.FP64)
    assert e.value.code == mpoevo.ESHAPE
    with pytest.raises(mpoevo.MpoevoError) as e:
        mpoevo.workspace_size(mpoevo.CALL_TRUNCATE, [2000, 5], mpoevo.FP64)
    assert e.value.code == mpoevo.ESHAPE
    # the one-site local tensor: its left block (Dbra_l d w_r Dket_r complex) and temporary at least
    one = [64, 64, 64, 64, 2, 6, 6]
    assert mpoevo.workspace_size(mpoevo.CALL_LOCAL_APPLY1, one, mpoevo.FP64) >= 2 * 64 * 2 * 6 * 64 * 16
    assert (mpoevo.workspace_size(mpoevo.CALL_LOCAL_APPLY1, one, mpoevo.FP32)
            < mpoevo.workspace_size(mpoevo.CALL_LOCAL_APPLY1, one, mpoevo.FP64))
    with pytest.raises(mpoevo.MpoevoError) as e:
        mpoevo.workspace_size(mpoevo.CALL_LOCAL_APPLY1, [64, 64, 0, 64, 2, 6, 6], mpoevo.FP32)
    assert e.value.code == mpoevo.ESHAPE


def test_device_calls_reject_null_handle():
    lib = mpoevo.load()
    assert lib.env_update(None, 0, 0, None, None, None, None, None, None, None, 0, None) == mpoevo.EINVAL
    assert lib.truncate(None, None, 1, 1, 1, 0.0, 0, None, None, None, None, None, None, None, 0, None) == mpoevo.EINVAL
    assert lib.step(None, None, None, None, None, None, 0, None) == mpoevo.EINVAL


def test_host_helpers_match_oracle():
    """The binding's purified MPO and splitting constants (host side, no GPU) against the
    oracle's own: the physical-leg operator of a purified chain and t1,2 = (1 +- i)/2."""
    rng = np.random.default_rng(21)
    for d in (2, 3):
        W = wl.complex_normal(rng, (3, d, d, 4))
        assert np.array_equal(mpoevo.purify_mpo(W), omp.purify(W))
    assert mpoevo.SPLIT_T1 == omp.SPLIT_T1 and mpoevo.SPLIT_T2 == omp.SPLIT_T2
    Wc, _ = mpoevo.mpo_build(*[getattr(wl.tfim_cylinder(4, 2.0), k) for k in ("A", "B", "C", "Dloc")], 2,
                             -0.1j, mpoevo.V2_EXTENDED)
    assert np.allclose(Wc, omp.build_mpo(wl.tfim_cylinder(4, 2.0), 2, -0.1j, "V2"), atol=1e-13)
