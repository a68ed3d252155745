"""Python binding of libmpoevo.so (ctypes): argument marshalling only.

Every computation runs in the library (host C++ for `mpo_build`, HIP kernels for the device
calls). PyTorch provides device memory and the current stream; the functions take torch
tensors on the GPU (complex128 for the FP64 path, complex64 for the FP32 path, see the header
include/mpoevo.h for layouts) and raise MpoevoError on any non-zero status.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpoevo.so")

OK, EINVAL, ESHAPE, ENOMEM, EHIP, ESOLVER, ENONFINITE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
FP64, FP32, BF16X3 = 0, 1, 2
V1_EXACT, V2_EXTENDED = 0, 1
LEFT, RIGHT = 0, 1
CALL_ENV_UPDATE, CALL_LOCAL_APPLY, CALL_TRUNCATE, CALL_STEP, CALL_EXPECTATION, CALL_STEP_BATCHED = 0, 1, 2, 3, 4, 5
CALL_LOCAL_APPLY1 = 6
TUNE_OFF, TUNE_ON, TUNE_FROZEN = 0, 1, 2
MAX_CHAINS = 4096
SVD_MAX_DIM = 1024


class MpoevoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mpoevo error {code}: {msg}")
        self.code = code


class _MPS(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int), ("d", ctypes.c_int), ("Dmax", ctypes.c_int),
                ("bond_dim", ctypes.POINTER(ctypes.c_int)), ("site", ctypes.POINTER(ctypes.c_void_p)),
                ("sector_table", ctypes.POINTER(ctypes.c_int)), ("phys_charge", ctypes.POINTER(ctypes.c_int))]


class _MPO(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int), ("d", ctypes.c_int), ("w", ctypes.POINTER(ctypes.c_int)),
                ("site", ctypes.POINTER(ctypes.c_void_p))]


class _Opts(ctypes.Structure):
    _fields_ = [("nsweeps", ctypes.c_int), ("prec", ctypes.c_int), ("cutoff", ctypes.c_double),
                ("input_right_canonical", ctypes.c_int), ("profile", ctypes.c_int),
                ("svd_cold_start", ctypes.c_int), ("nsites", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("guess", ctypes.c_int)]


MAX_KERNEL_STATS = 16
KERNEL_KINDS = ("jacobi_svd", "complex_gemm", "w_contraction", "householder_qr")


class _KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 224), ("kind", ctypes.c_int), ("split_k", ctypes.c_int),
                ("launches", ctypes.c_int), ("ms", ctypes.c_double), ("work", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_double), ("discarded_max", ctypes.c_double),
                ("discarded_sum", ctypes.c_double), ("visits", ctypes.c_int),
                ("max_bond", ctypes.c_int), ("gflop", ctypes.c_double), ("svd_sweeps_max", ctypes.c_int),
                ("t_jacobi_ms", ctypes.c_double), ("jacobi_gflop", ctypes.c_double), ("n_jacobi", ctypes.c_int),
                ("t_gemm_ms", ctypes.c_double), ("gemm_gflop", ctypes.c_double), ("n_gemm", ctypes.c_int),
                ("t_wmix_ms", ctypes.c_double), ("wmix_gbyte", ctypes.c_double), ("n_wmix", ctypes.c_int),
                ("svd_sweeps_total", ctypes.c_int), ("svd_sweeps_hist", ctypes.c_int * 32),
                ("n_kernel_stats", ctypes.c_int), ("kernel_stats", _KernelStat * MAX_KERNEL_STATS),
                ("graph", ctypes.c_int), ("guess", ctypes.c_int), ("one_site_visits", ctypes.c_int),
                ("two_site_redo", ctypes.c_int)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the library once (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise MpoevoError(EUNSUPPORTED, f"{path} is missing: run paper_2302_14181_amd.build first")
    lib = ctypes.CDLL(path, mode=os.RTLD_LOCAL | os.RTLD_NOW)
    vp, ip, dp, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), ctypes.c_size_t
    lib.mpoevo_version.restype = ctypes.c_char_p
    lib.mpoevo_last_error.restype = ctypes.c_char_p
    lib.mpoevo_last_error.argtypes = [vp]
    lib.mpoevo_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.mpoevo_destroy.argtypes = [vp]
    lib.mpoevo_check_solver.argtypes = [vp, ip]
    lib.mpo_build.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, ctypes.c_int, ctypes.c_double,
                              ctypes.c_double, ctypes.c_int, ip, ip, ip, dp, sz, ip]
    lib.mpoevo_workspace_size.argtypes = [ctypes.c_int, ip, ctypes.c_int, ctypes.POINTER(sz)]
    lib.env_update.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp, ip, vp, sz, vp]
    lib.local_apply.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, ip, vp, sz, vp]
    lib.truncate.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                             vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.step.argtypes = [vp, ctypes.POINTER(_MPS), ctypes.POINTER(_MPO), ctypes.POINTER(_Opts),
                         ctypes.POINTER(_Stats), vp, sz, vp]
    lib.expectation.argtypes = [vp, ctypes.POINTER(_MPS), ctypes.POINTER(_MPO), ctypes.c_int, ctypes.c_int,
                                vp, vp, sz, vp]
    lib.step_batched.argtypes = [vp, ctypes.c_int, ctypes.POINTER(_MPS), ctypes.POINTER(_MPO),
                                 ctypes.POINTER(_Opts), ctypes.POINTER(_Stats), vp, sz, vp]
    lib.overlap.argtypes = [vp, ctypes.POINTER(_MPS), ctypes.POINTER(_MPO), ctypes.POINTER(_MPS), ctypes.c_int,
                            ctypes.c_int, vp, vp, sz, vp]
    lib.env_update_noalloc.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp, ip, vp]
    lib.mpoevo_set_tuning.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.mpoevo_product_plan.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ip, ip]
    for name in ("mpoevo_create", "mpoevo_destroy", "mpoevo_check_solver", "mpo_build",
                 "mpoevo_workspace_size", "env_update", "local_apply", "truncate", "step", "expectation",
                 "step_batched", "mpoevo_set_tuning", "mpoevo_product_plan", "env_update_noalloc", "overlap"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def exported_symbols():
    return ["mpoevo_create", "mpoevo_destroy", "mpoevo_last_error", "mpoevo_version", "mpo_build",
            "env_update", "local_apply", "truncate", "mpoevo_check_solver", "step",
            "expectation", "step_batched", "mpoevo_workspace_size", "mpoevo_set_tuning",
            "mpoevo_product_plan", "env_update_noalloc", "overlap"]


def _check(rc: int, handle=None):
    if rc != OK:
        lib = load()
        msg = lib.mpoevo_last_error(handle.ptr if handle is not None else None)
        raise MpoevoError(rc, msg.decode() if msg else "")


def _iarr(values):
    return (ctypes.c_int * len(values))(*[int(v) for v in values])


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ------------------------------------------------------------------------------------ host
def mpo_build(A, B, C, Dloc, order: int, tau: complex, variant: int = V2_EXTENDED,
              inner_charge=None, phys_charge=None):
    """Order-N MPO W[w][d][d][w] (numpy complex128) and, with charges, the level charges."""
    lib = load()
    A = np.ascontiguousarray(A, dtype=np.complex128)
    B = np.ascontiguousarray(B, dtype=np.complex128)
    C = np.ascontiguousarray(C, dtype=np.complex128)
    D = np.ascontiguousarray(Dloc, dtype=np.complex128)
    d, chi = D.shape[0], B.shape[0]
    qi = _iarr(inner_charge) if inner_charge is not None else None
    qp = _iarr(phys_charge) if phys_charge is not None else None
    w = ctypes.c_int(0)
    args = (d, chi, _dptr(A.view(np.float64)), _dptr(B.view(np.float64)), _dptr(C.view(np.float64)),
            _dptr(D.view(np.float64)), order, float(np.real(tau)), float(np.imag(tau)), variant, qi, qp)
    _check(lib.mpo_build(*args, ctypes.byref(w), None, 0, None))
    W = np.zeros((w.value, d, d, w.value), dtype=np.complex128)
    lc = (ctypes.c_int * w.value)() if qi is not None else None
    _check(lib.mpo_build(*args, ctypes.byref(w), _dptr(W.view(np.float64)), W.size, lc))
    return W, (np.array(list(lc), dtype=np.int64) if lc is not None else None)


def workspace_size(call_id: int, dims, prec: int) -> int:
    lib = load()
    out = ctypes.c_size_t(0)
    _check(lib.mpoevo_workspace_size(call_id, _iarr(dims), prec, ctypes.byref(out)))
    return out.value


# ---------------------------------------------------------------------------------- device
def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _prec_of(t, prec=None) -> int:
    """Precision of a call on tensors of t's dtype: complex128 -> FP64; complex64 -> FP32, or
    BF16X3 when asked for (the same complex64 storage, split-bf16 products)."""
    torch = _torch()
    if t.dtype == torch.complex128:
        if prec not in (None, FP64):
            raise MpoevoError(EINVAL, "complex128 tensors take the FP64 path")
        return FP64
    if t.dtype == torch.complex64:
        if prec not in (None, FP32, BF16X3):
            raise MpoevoError(EINVAL, "complex64 tensors take the FP32 or BF16X3 path")
        return FP32 if prec is None else prec
    raise MpoevoError(EINVAL, f"unsupported dtype {t.dtype}")


def _workspace(nbytes: int, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class Handle:
    """Library handle on one HIP device."""

    def __init__(self, device: int = 0):
        lib = load()
        self.ptr = ctypes.c_void_p()
        _check(lib.mpoevo_create(ctypes.byref(self.ptr), device))
        self.device = device

    def close(self):
        if self.ptr:
            load().mpoevo_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, mode: int, clear: bool = False):
        """Tile choice of the products (TUNE_OFF: fixed rule; TUNE_ON: time the candidate plans
        of each new shape; TUNE_FROZEN: keep the tuned shapes, tune no more)."""
        _check(load().mpoevo_set_tuning(self.ptr, int(mode), int(bool(clear))), self)

    def product_plan(self, prec: int, M: int, N: int, K: int, batch: int = 1) -> dict:
        """Plan of a product of that shape on this handle: tile, K splits, tuned or not."""
        out = (ctypes.c_int * 4)()
        n = ctypes.c_int(0)
        _check(load().mpoevo_product_plan(self.ptr, prec, M, N, K, batch, out, ctypes.byref(n)), self)
        return {"tile": (out[0], out[1]), "splits": out[2], "tuned": bool(out[3]), "entries": n.value}

    def check_solver(self) -> int:
        """Raise if an SVD since the last check failed; return the largest Jacobi sweep count."""
        sweeps = ctypes.c_int(0)
        _check(load().mpoevo_check_solver(self.ptr, ctypes.byref(sweeps)), self)
        return sweeps.value


def env_update(h: Handle, side: int, E_in, bra, W, ket, E_out, workspace=None, stream=None,
               prec=None):
    """Environment update (see include/mpoevo.h). Tensors: E (Dbra, w, Dket), bra/ket
    (D_l, d, D_r), W (w_l, d, d, w_r), all complex128 or all complex64 on the device;
    prec=BF16X3 selects split-bf16 products for complex64 tensors."""
    prec = _prec_of(E_in, prec)
    Dbl, d, Dbr = bra.shape
    Dkl, _, Dkr = ket.shape
    wl, _, _, wr = W.shape
    dims = [Dbl, Dkl, Dbr, Dkr, d, wl, wr]
    if workspace is None:
        workspace = _workspace(workspace_size(CALL_ENV_UPDATE, dims, prec), E_in.device)
    _check(load().env_update(h.ptr, side, prec, _ptr(E_in), _ptr(bra), _ptr(W), _ptr(ket), _ptr(E_out),
                             _iarr(dims), _ptr(workspace), workspace.numel(), _stream(stream)), h)


NOALLOC_SCRATCH_BYTES = 64 << 20


def env_update_noalloc(h: Handle, side: int, E_in, bra, W, ket, E_out, stream=None, prec=None):
    """env_update without a workspace: the library's per-device scratch holds the intermediates
    (for callers that cannot allocate; calls overlapping on one device race)."""
    prec = _prec_of(E_in, prec)
    Dbl, d, Dbr = bra.shape
    Dkl, _, Dkr = ket.shape
    wl, _, _, wr = W.shape
    dims = [Dbl, Dkl, Dbr, Dkr, d, wl, wr]
    _check(load().env_update_noalloc(h.ptr, side, prec, _ptr(E_in), _ptr(bra), _ptr(W), _ptr(ket),
                                     _ptr(E_out), _iarr(dims), _stream(stream)), h)


def local_apply(h: Handle, Lenv, W1, W2, M1, M2, Renv, Theta, workspace=None, stream=None,
                prec=None):
    """Projected two-site tensor into Theta (complex128, (Dbra_l*d) x (d*Dbra_r)); prec as for
    env_update."""
    prec = _prec_of(Lenv, prec)
    Dbl, wl, Dkl = Lenv.shape
    Dkm = M1.shape[2]
    Dkr = M2.shape[2]
    Dbr, wr, _ = Renv.shape
    d = M1.shape[1]
    wm = W1.shape[3]
    dims = [Dbl, Dkl, Dkm, Dkr, Dbr, d, wl, wm, wr]
    if workspace is None:
        workspace = _workspace(workspace_size(CALL_LOCAL_APPLY, dims, prec), Lenv.device)
    _check(load().local_apply(h.ptr, 2, prec, _ptr(Lenv), _ptr(W1), _ptr(W2), _ptr(M1), _ptr(M2),
                              _ptr(Renv), _ptr(Theta), _iarr(dims), _ptr(workspace), workspace.numel(),
                              _stream(stream)), h)


def local_apply_one_site(h: Handle, Lenv, W, M, Renv, Theta, workspace=None, stream=None, prec=None):
    """Projected one-site tensor into Theta (complex128, (Dbra_l*d) x Dbra_r); prec as for
    env_update."""
    prec = _prec_of(Lenv, prec)
    Dbl, wl, Dkl = Lenv.shape
    Dbr, wr, Dkr = Renv.shape
    d = M.shape[1]
    dims = [Dbl, Dkl, Dkr, Dbr, d, wl, wr]
    if workspace is None:
        workspace = _workspace(workspace_size(CALL_LOCAL_APPLY1, dims, prec), Lenv.device)
    _check(load().local_apply(h.ptr, 1, prec, _ptr(Lenv), _ptr(W), None, _ptr(M), None, _ptr(Renv),
                              _ptr(Theta), _iarr(dims), _ptr(workspace), workspace.numel(), _stream(stream)), h)


def truncate(h: Handle, Theta, Dmax: int, cutoff: float, direction: int, A_out, B_out,
             k=None, discarded=None, norm=None, sigma=None, workspace=None, stream=None):
    """FP64 SVD truncation of Theta (m x n complex128); outputs A_out (m x kcap), B_out
    (kcap x n); optional device scalars k (int32), discarded, norm (float64), sigma."""
    m, n = Theta.shape
    if workspace is None:
        workspace = _workspace(workspace_size(CALL_TRUNCATE, [m, n], FP64), Theta.device)
    _check(load().truncate(h.ptr, _ptr(Theta), m, n, Dmax, cutoff, direction, _ptr(A_out), _ptr(B_out),
                           _ptr(k), _ptr(discarded), _ptr(norm), _ptr(sigma), _ptr(workspace),
                           workspace.numel(), _stream(stream)), h)


@dataclass
class StepStats:
    norm: float
    discarded_max: float
    discarded_sum: float
    visits: int
    max_bond: int
    gflop: float
    svd_sweeps_max: int
    profile: dict | None = None
    svd_sweeps_total: int = 0
    svd_sweeps_hist: tuple = ()
    graph: int = 0  # use_graph: 0 issued launch by launch, 1 captured into a new graph, 2 replayed
    guess: int = 0  # the guess the sweeps started from: 0 psi, 1 the zip-up
    one_site_visits: int = 0  # visits that took the one-site update
    two_site_redo: int = 0  # 1: the automatic mode's mixed sweep was redone with two-site updates


class DeviceMPS:
    """MPS on the device: complex128 site buffers of capacity Dmax * d * Dmax, bonds on the host.
    U(1) chains: charges[b] lists the charge of every index of bond b (nondecreasing; the sites'
    bond indices in charge order) and phys_charge that of every physical index; a step then runs
    the U(1) fit and updates self.charges."""

    def __init__(self, sites, Dmax: int, device="cuda", charges=None, phys_charge=None):
        torch = _torch()
        self.L = len(sites)
        self.d = sites[0].shape[1]
        self.Dmax = Dmax
        self.bond = [1] + [int(s.shape[2]) for s in sites]
        self.charges = None
        self.phys_charge = None
        if charges is not None:
            if phys_charge is None or len(charges) != self.L + 1:
                raise MpoevoError(EINVAL, "charges need L + 1 bonds and phys_charge")
            self.charges = [list(map(int, c)) for c in charges]
            self.phys_charge = list(map(int, phys_charge))
            if [len(c) for c in self.charges] != self.bond:
                raise MpoevoError(ESHAPE, "charges must list every bond index")
        cap = Dmax * self.d * Dmax
        self.buf = []
        for s in sites:
            if s.shape[0] > Dmax or s.shape[2] > Dmax:
                raise MpoevoError(ESHAPE, "site bond exceeds Dmax")
            t = torch.zeros(cap, dtype=torch.complex128, device=device)
            flat = torch.from_numpy(np.ascontiguousarray(s, dtype=np.complex128).reshape(-1))
            t[: flat.numel()].copy_(flat)
            self.buf.append(t)

    def to_numpy(self):
        out = []
        for i, t in enumerate(self.buf):
            a, b = self.bond[i], self.bond[i + 1]
            out.append(t[: a * self.d * b].cpu().numpy().reshape(a, self.d, b).copy())
        return out


class DeviceMPO:
    """Per-site MPO tensors on the device (complex128)."""

    def __init__(self, Ws, device="cuda"):
        torch = _torch()
        self.L = len(Ws)
        self.d = Ws[0].shape[1]
        self.w = [int(Ws[0].shape[0])] + [int(W.shape[3]) for W in Ws]
        cache = {}
        self.buf = []
        for W in Ws:
            key = id(W)
            if key not in cache:
                cache[key] = torch.from_numpy(np.ascontiguousarray(W, dtype=np.complex128)).to(device)
            self.buf.append(cache[key])


def _c_mps(mps: DeviceMPS):
    """ctypes view of a DeviceMPS: (structure, bond array, sector table array or None, keep-alive)."""
    bond = _iarr(mps.bond)
    sites = (ctypes.c_void_p * mps.L)(*[t.data_ptr() for t in mps.buf])
    table = qp = None
    if mps.charges is not None:
        flat = [0] * ((mps.L + 1) * mps.Dmax)
        for b, c in enumerate(mps.charges):
            flat[b * mps.Dmax:b * mps.Dmax + len(c)] = c
        table = _iarr(flat)
        qp = _iarr(mps.phys_charge)
    return _MPS(mps.L, mps.d, mps.Dmax, bond, sites, table, qp), bond, table, (sites, qp)


def _c_mps_update(mps: DeviceMPS, bond, table):
    mps.bond = [bond[i] for i in range(mps.L + 1)]
    if table is not None:
        mps.charges = [[table[b * mps.Dmax + j] for j in range(mps.bond[b])] for b in range(mps.L + 1)]


def step_workspace(mps: DeviceMPS, mpo: DeviceMPO, prec: int):
    dims = [mps.L, mps.d, mps.Dmax, max(mpo.w)]
    return _workspace(workspace_size(CALL_STEP, dims, prec), mps.buf[0].device)


def _default_step_workspace(h: "Handle", mps: DeviceMPS, mpo: DeviceMPO, prec: int):
    """The workspace of step calls made without one: kept alive on the MPS object per handle,
    precision and MPO bond, so that the truncation preconditioners a step leaves in it stay
    intact until the next step (a temporary would return to the allocator and be handed out
    again between the calls)."""
    cache = mps.__dict__.setdefault("_step_ws", {})
    key = (h.ptr.value, prec, max(mpo.w))
    ws = cache.get(key)
    if ws is None:
        ws = cache[key] = step_workspace(mps, mpo, prec)
    return ws


NSITES_AUTO = -1  # step option: one-site updates once every bond is at its largest value
# step option guess: psi (right-canonicalised), the zip-up of W psi, or the zip-up while bonds grow
GUESS_AUTO, GUESS_CANONICAL, GUESS_ZIPUP = -1, 0, 1


def step(h: Handle, mps: DeviceMPS, mpo: DeviceMPO, nsweeps: int = 2, prec: int = FP64,
         cutoff: float = 1e-14, input_right_canonical: bool = False, workspace=None,
         stream=None, profile=False, svd_cold_start: bool = False, nsites: int = 2,
         use_graph: bool = False, guess: int = 0) -> StepStats:
    """One time step of the variational fit; mps is updated in place (see include/mpoevo.h).
    profile: False, True (time every kernel class) or PROFILE_JACOBI (the Jacobi kernel only).
    Without a workspace the MPS object's own default workspace is used (kept between calls)."""
    if workspace is None:
        workspace = _default_step_workspace(h, mps, mpo, prec)
    cm, bond, table, _keep = _c_mps(mps)
    wsites = (ctypes.c_void_p * mpo.L)(*[t.data_ptr() for t in mpo.buf])
    cw = _MPO(mpo.L, mpo.d, _iarr(mpo.w), wsites)
    opts = _Opts(nsweeps, prec, cutoff, int(bool(input_right_canonical)), _profile_code(profile),
                 int(bool(svd_cold_start)), int(nsites), int(bool(use_graph)),
                 int(guess))
    st = _Stats()
    _check(load().step(h.ptr, ctypes.byref(cm), ctypes.byref(cw), ctypes.byref(opts), ctypes.byref(st),
                       _ptr(workspace), workspace.numel(), _stream(stream)), h)
    _c_mps_update(mps, bond, table)
    return _stats_of(st, profile)


PROFILE_JACOBI = 2  # step option: time the Jacobi kernel only (least host overhead)

# Splitting composite (Sec. 8.3, splitting schemes): first-order operators at the complex steps
# t1 tau and t2 tau, t1,2 = (1 +- i)/2, applied one after the other are accurate to second order.
SPLIT_T1 = (1 + 1j) / 2
SPLIT_T2 = (1 - 1j) / 2


def purify_mpo(W: np.ndarray) -> np.ndarray:
    """MPO site tensor of O acting on the physical leg of a purified chain (finite temperature:
    the state exp(-beta H / 2) applied to the beta = 0 product of maximally entangled pairs gives
    thermal averages; cf. the exp(-beta H) construction of Sec. 8.4). Local index s d + a, the
    ancilla a fastest: W'[alpha, s' d + a, s d + a, beta] = W[alpha, s', s, beta]."""
    w, d, _, w2 = W.shape
    out = np.zeros((w, d * d, d * d, w2), dtype=np.complex128)
    for a in range(d):
        out[:, a::d, a::d, :] = W
    return out


def split_step(h: Handle, mps: DeviceMPS, first: DeviceMPO, second: DeviceMPO, nsweeps: int = 2,
               prec: int = FP64, cutoff: float = 1e-14, input_right_canonical: bool = False,
               workspace=None, stream=None) -> tuple:
    """One step of a splitting composite: the fit of `first` applied to mps, then the fit of
    `second` applied to the result (two step calls; the first leaves mps right-canonical). For the
    second-order composite pass the first-order MPOs at SPLIT_T2 * tau and SPLIT_T1 * tau (their
    product is the same operator to second order in either order). Returns both StepStats; the
    product of their norms is the norm of the composite applied to mps."""
    if workspace is None:
        workspace = _default_step_workspace(h, mps, first if max(first.w) >= max(second.w) else second, prec)
    a = step(h, mps, first, nsweeps=nsweeps, prec=prec, cutoff=cutoff,
             input_right_canonical=input_right_canonical, workspace=workspace, stream=stream)
    b = step(h, mps, second, nsweeps=nsweeps, prec=prec, cutoff=cutoff, input_right_canonical=True,
             workspace=workspace, stream=stream)
    return a, b


def _profile_code(profile) -> int:
    if profile is True or profile == 1:
        return 1
    if profile == PROFILE_JACOBI:
        return PROFILE_JACOBI
    if not profile:
        return 0
    raise ValueError("profile must be False, True or PROFILE_JACOBI")


def _stats_of(st, profile) -> StepStats:
    prof = None
    if profile:
        prof = {k: getattr(st, k) for k in ("t_jacobi_ms", "jacobi_gflop", "n_jacobi", "t_gemm_ms",
                                            "gemm_gflop", "n_gemm", "t_wmix_ms", "wmix_gbyte", "n_wmix")}
        prof["kernels"] = [{"name": k.name.decode(errors="replace"), "kind": KERNEL_KINDS[k.kind],
                            "split_k": bool(k.split_k), "launches": k.launches, "ms": k.ms, "work": k.work}
                           for k in st.kernel_stats[:st.n_kernel_stats]]
    return StepStats(st.norm, st.discarded_max, st.discarded_sum, st.visits, st.max_bond, st.gflop,
                     st.svd_sweeps_max, prof, st.svd_sweeps_total, tuple(st.svd_sweeps_hist), st.graph,
                     st.guess, st.one_site_visits, st.two_site_redo)


def step_batched_workspace(chains, mpos, prec: int):
    dims = [len(chains)]
    for mps, mpo in zip(chains, mpos):
        dims += [mps.L, mps.d, mps.Dmax, max(mpo.w)]
    return _workspace(workspace_size(CALL_STEP_BATCHED, dims, prec), chains[0].buf[0].device)


def step_batched(h: Handle, chains, mpos, nsweeps: int = 2, prec: int = FP64, cutoff: float = 1e-14,
                 input_right_canonical: bool = False, workspace=None, stream=None, profile: bool = False,
                 svd_cold_start: bool = False, nsites: int = 2, use_graph: bool = False, guess: int = 0):
    """One time step of every chain (lists of DeviceMPS and DeviceMPO of equal length), advanced
    concurrently by the library; each MPS is updated in place. Returns one StepStats per chain."""
    if len(chains) != len(mpos) or not chains:
        raise MpoevoError(EINVAL, "step_batched: need equal, non-empty lists of chains and MPOs")
    if workspace is None:
        workspace = step_batched_workspace(chains, mpos, prec)
    n = len(chains)
    keep = []  # ctypes arrays referenced by the structures
    cms = (_MPS * n)()
    cws = (_MPO * n)()
    tables = []
    for c, (mps, mpo) in enumerate(zip(chains, mpos)):
        cm, bond, table, k2 = _c_mps(mps)
        w = _iarr(mpo.w)
        wsites = (ctypes.c_void_p * mpo.L)(*[t.data_ptr() for t in mpo.buf])
        keep += [bond, k2, w, wsites]
        tables.append(table)
        cms[c] = cm
        cws[c] = _MPO(mpo.L, mpo.d, w, wsites)
    opts = _Opts(nsweeps, prec, cutoff, int(bool(input_right_canonical)), _profile_code(profile),
                 int(bool(svd_cold_start)), int(nsites), int(bool(use_graph)),
                 int(guess))
    st = (_Stats * n)()
    _check(load().step_batched(h.ptr, n, cms, cws, ctypes.byref(opts), st, _ptr(workspace),
                               workspace.numel(), _stream(stream)), h)
    for c, mps in enumerate(chains):
        _c_mps_update(mps, keep[4 * c], tables[c])
    return [_stats_of(st[c], profile) for c in range(n)]


def expectation(h: Handle, mps: DeviceMPS, mpo: DeviceMPO, left: int = 0, right: int = 0,
                workspace=None, stream=None) -> complex:
    """<psi| l.O_1...O_L.r |psi> on the device in FP64 (see include/mpoevo.h); waits for the result."""
    torch = _torch()
    dev = mps.buf[0].device
    if workspace is None:
        workspace = _workspace(workspace_size(CALL_EXPECTATION, [mps.L, mps.d, mps.Dmax, max(mpo.w)], FP64), dev)
    cm, bond, table, _keep = _c_mps(mps)
    wsites = (ctypes.c_void_p * mpo.L)(*[t.data_ptr() for t in mpo.buf])
    cw = _MPO(mpo.L, mpo.d, _iarr(mpo.w), wsites)
    out = torch.zeros(2, dtype=torch.float64, device=dev)
    _check(load().expectation(h.ptr, ctypes.byref(cm), ctypes.byref(cw), left, right, _ptr(out),
                              _ptr(workspace), workspace.numel(), _stream(stream)), h)
    (stream if stream is not None else torch.cuda.current_stream()).synchronize()
    v = out.cpu().numpy()
    return complex(v[0], v[1])


def overlap(h: Handle, bra: DeviceMPS, mpo: DeviceMPO, ket: DeviceMPS, left: int = 0, right: int = 0,
            workspace=None, stream=None) -> complex:
    """<bra| l.O_1...O_L.r |ket> on the device in FP64 (see include/mpoevo.h); waits for the result."""
    torch = _torch()
    dev = ket.buf[0].device
    Dm = max(bra.Dmax, ket.Dmax)
    if workspace is None:
        workspace = _workspace(workspace_size(CALL_EXPECTATION, [ket.L, ket.d, Dm, max(mpo.w)], FP64), dev)
    cb, _, _, kb = _c_mps(bra)
    ck, _, _, kk = _c_mps(ket)
    wsites = (ctypes.c_void_p * mpo.L)(*[t.data_ptr() for t in mpo.buf])
    cw = _MPO(mpo.L, mpo.d, _iarr(mpo.w), wsites)
    out = torch.zeros(2, dtype=torch.float64, device=dev)
    _check(load().overlap(h.ptr, ctypes.byref(cb), ctypes.byref(cw), ctypes.byref(ck), left, right, _ptr(out),
                          _ptr(workspace), workspace.numel(), _stream(stream)), h)
    (stream if stream is not None else torch.cuda.current_stream()).synchronize()
    v = out.cpu().numpy()
    return complex(v[0], v[1])
