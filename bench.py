"""Benchmark: seconds per time step of the variational higher-order MPO evolution on one MI355X.

Workload (default): the quench of the open transverse-field Ising chain H = -sum Z Z - g sum X,
L = 64, from the ground state at g = 0.5 (tests/golden/tfim_g05_L64_ground.npz, prepared by the
oracle) to g = 1.5, with the order-2 extended MPO (w = 3) of exp(-i tau H), tau = 0.1, bond
dimension D <= 128, truncation cutoff 1e-14 sigma_1, two sweeps per step: K time steps from t = 0
(default K = 100, the whole run). The bond dimension grows from about 24 to 128 during the first
twenty steps and stays at 128 afterwards. Contractions run on the FP32 matrix cores, the SVD
truncation in FP64. `value` is the mean seconds per step over the K timed steps (HIP events on
the launch stream, bracketed by device synchronisation); W untimed warm-up steps run first on a
separate copy of the initial state.

Also reported: the same opening steps on the plain FP64 path (FP32/FP64 time ratio on identical
steps), one step at saturated bond dimension on a seeded random MPS (D = 128 on every bulk bond;
also on the FP64 path, for the ratio at saturation),
one step of the long-range chain at D = 256 with the w = 271 order-3 MPO on the FP32, FP64 and
split-BF16x3 paths (step time and matrix-core rate of the contractions: the "TFLOP/s at D = 256"
part of the metric),
the environment-update microbenchmark at D = 256, d = 2, w = 8 (the matrix-core roofline target),
the Jacobi kernel's time summed over the timed steps (HIP events around its launches only, the
roofline line) and every kernel class on one extra saturated step, per-step parity of the first step against the
oracle from the same initial state on each path (infidelity and <Z_32> error), and the CPU oracle timed on one
saturated-bond step (the cpu_baseline).

With --workload lr3: the long-range Ising chain of the configuration with the largest MPO bond,
J(r) = r^-2 as six exponentials (tests/golden/lr_fit_K6.json), g = 1, L = 100, order-3 extended MPO
(w = 271), tau = 0.1, at saturated bond dimension D = 256 (seeded random MPS), K timed steps after
W warm-up steps of the same trajectory (defaults K = 2, W = 1), FP32 and FP64 paths; the CPU oracle
is timed on one bond visit of that workload and scaled to a step (labelled extrapolated).

With --workload batched: 64 independent TFIM chains (g ~ U(0.5, 1.5), L in {32, 64, 96, 128},
D in {32, 64, 128, 256}, seed 2), order-2 extended MPO, tau = 0.1, from all-up, K steps (default 3)
advanced together by step_batched, against the same steps taken chain by chain; the oracle checks
and times the first step of the first four chains.

With --workload split: the quench above advanced by the splitting composite of Sec. 8.3 (the
first-order MPO at t2 tau, then at t1 tau, t1,2 = (1 +- i)/2: two fits per step at MPO bond 2)
against the order-2 MPO (one fit at bond 3), K steps each (default 20) from the same state.

With --workload thermal: finite temperature by purification on the L = 64 TFIM at g = 1 (physical
and ancilla leg per site, d = 4): the order-2 MPO at tau = -0.05 on the physical legs, K steps
(default 20) from beta = 0 (maximally entangled pairs) to beta = 2 K 0.05, D <= 128; FP32 and
FP64 paths, energy per site at the end from the device expectation.

With --workload cylinder: the efficiency set-up of Sec. 8.2 on a finite W = 4 spiral cylinder
(TFIM, h = 2, 8 x 4 = 32 sites, D <= 64): a ground state by imaginary-time steps, a spin flip on
the middle site, evolution to T = 1 with orders 1-3 at dt = 0.2, 0.1, 0.05, and the fidelity
density against an order-3 run at dt = 0.0125 (standing in for the TDVP reference).

With --workload env: only the left environment update at D = 256, d = 2, w = 8 (the matrix-core
roofline case), K calls per precision (default 100) timed with HIP events on the launch stream.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec fp32|fp64|bf16x3] [--fp64-steps N]
                       [--no-cpu] [--no-fp64] [--workload quench|lr3|batched|env|split|thermal|cylinder]
                       [--order 1|2|3|4] [--tau T] [--progress]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3e12
PEAK_FP64_MFMA = 78.6e12
PEAK_BF16_MFMA = 2.5e15
# split-BF16x3 issues three bf16 products per algorithmic one
CEIL_BF16X3 = PEAK_BF16_MFMA / 3
PEAK_FP64_VALU = 78.6e12
PEAK_HBM = 8.0e12
DTYPES = {"fp32": "f32 contractions, f64 SVD", "fp64": "f64",
          "bf16x3": "split-bf16x3 contractions (f32 storage, f32 accumulation), f64 SVD"}
GROUND = os.path.join(ROOT, "tests", "golden", "tfim_g05_L64_ground.npz")
L, D, G_AFTER, ORDER, TAU = 64, 128, 1.5, 2, 0.1


def prec_of(mp, name: str) -> int:
    return {"fp32": mp.FP32, "fp64": mp.FP64, "bf16x3": mp.BF16X3}[name]


def env_microbench(mp, h, torch, prec: int, reps: int = 50):
    """Time env_update (left) at D = 256, d = 2, w = 8 with HIP events on the launch stream."""
    from paper_2302_14181_amd import workloads as wl
    E, M, N, W = wl.env_microbench_inputs(0)
    dt = torch.complex128 if prec == mp.FP64 else torch.complex64
    t = {k: torch.from_numpy(v).to(dt).cuda() for k, v in dict(E=E, M=M, N=N, W=W).items()}
    out = torch.empty((256, 8, 256), dtype=dt, device="cuda")
    ws = torch.empty(mp.workspace_size(mp.CALL_ENV_UPDATE, [256, 256, 256, 256, 2, 8, 8], prec),
                     dtype=torch.uint8, device="cuda")
    for _ in range(3):
        mp.env_update(h, mp.LEFT, t["E"], t["N"], t["W"], t["M"], out, workspace=ws, prec=prec)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        mp.env_update(h, mp.LEFT, t["E"], t["N"], t["W"], t["M"], out, workspace=ws, prec=prec)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    Dm, d, w = 256, 2, 8
    flop = 8.0 * (2 * Dm ** 3 * d * w + Dm ** 2 * d ** 2 * w ** 2)
    return ms, flop


def load_ground():
    z = np.load(GROUND)
    return [z[f"site_{i:03d}"] for i in range(L)]


def run_lr3(args, torch, mp, wl, h, steps=None, warmup=None, embedded=False):
    """K steps of the order-3 long-range Ising chain at D = 256 (w = 271): the chosen path, and
    with an FP32 path also plain FP64 and split-BF16x3 on the same steps.
    embedded: return a summary dict (FP32 vs FP64 vs BF16X3 step time and product rate)."""
    import json as _json
    Llr, Dlr, order, tau = 100, 256, 3, 0.1
    if steps is None:
        steps = args.steps if args.steps != 100 else 2
    if warmup is None:
        warmup = args.warmup
    fit = _json.load(open(os.path.join(ROOT, "tests", "golden", "lr_fit_K6.json")))
    H = wl.lr_ising(np.array(fit["coeffs"]), np.array(fit["lambdas"]), 1.0)
    W, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, order, -1j * tau, mp.V2_EXTENDED)
    w = W.shape[0]
    dw = mp.DeviceMPO([W] * Llr)
    psi = wl.random_mps(np.random.default_rng(0), Llr, 2, Dlr)

    def run(p, n):
        dm = mp.DeviceMPS(psi, Dmax=Dlr)
        ws = mp.step_workspace(dm, dw, p)
        for k in range(warmup):
            mp.step(h, dm, dw, prec=p, input_right_canonical=k > 0, workspace=ws)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
        ev[0].record()
        st = []
        for k in range(n):
            st.append(mp.step(h, dm, dw, prec=p, input_right_canonical=(warmup + k) > 0, workspace=ws,
                              profile=True))
            ev[k + 1].record()
        torch.cuda.synchronize()
        ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(n)]
        del ws, dm
        torch.cuda.empty_cache()
        return ms, st

    prec = mp.FP32 if embedded else prec_of(mp, args.prec)
    ms, st = run(prec, steps)
    sec = float(np.sum(ms)) / 1e3 / steps
    prof = {k: float(sum(x.profile[k] for x in st)) for k in st[0].profile}
    peak = {mp.FP32: PEAK_FP32_MFMA, mp.FP64: PEAK_FP64_MFMA, mp.BF16X3: CEIL_BF16X3}[prec]
    gemm_tf = prof["gemm_gflop"] / prof["t_gemm_ms"] if prof["t_gemm_ms"] > 0 else 0.0
    fp64 = bf = None
    if (embedded or not args.no_fp64) and prec == mp.FP32:
        ms64, st64 = run(mp.FP64, steps)
        p64 = {k: float(sum(x.profile[k] for x in st64)) for k in st64[0].profile}
        fp64 = {"fp64_s_per_step": float(np.sum(ms64)) / 1e3 / steps,
                "fp64_gemm_tflops": p64["gemm_gflop"] / p64["t_gemm_ms"] if p64["t_gemm_ms"] > 0 else 0.0}
        fp64["fp32_speedup"] = fp64["fp64_s_per_step"] / sec
        msb, stb = run(mp.BF16X3, steps)
        pb = {k: float(sum(x.profile[k] for x in stb)) for k in stb[0].profile}
        bf = {"bf16x3_s_per_step": float(np.sum(msb)) / 1e3 / steps,
              "bf16x3_gemm_tflops": pb["gemm_gflop"] / pb["t_gemm_ms"] if pb["t_gemm_ms"] > 0 else 0.0}
        bf["bf16x3_frac_of_ceiling"] = bf["bf16x3_gemm_tflops"] * 1e12 / CEIL_BF16X3
        bf["bf16x3_speedup_vs_fp64"] = fp64["fp64_s_per_step"] / bf["bf16x3_s_per_step"]
    if embedded:
        return {"workload": f"long-range Ising L={Llr}, order-{order} extended MPO (w={w}), tau={tau}, "
                            f"D={Dlr} saturated random MPS, {steps} step(s) after {warmup} warm-up",
                "fp32_s_per_step": sec, "fp64_s_per_step": fp64["fp64_s_per_step"],
                "fp32_speedup": fp64["fp32_speedup"], "step_tflop": float(np.mean([x.gflop for x in st])) / 1e3,
                "fp32_gemm_tflops": gemm_tf, "fp32_gemm_frac_of_mfma_peak": gemm_tf * 1e12 / PEAK_FP32_MFMA,
                "fp64_gemm_tflops": fp64["fp64_gemm_tflops"],
                "fp64_gemm_frac_of_mfma_peak": fp64["fp64_gemm_tflops"] * 1e12 / PEAK_FP64_MFMA,
                "jacobi_share_fp32": prof["t_jacobi_ms"] / max(float(np.sum(ms)), 1e-9),
                "bf16x3": bf}
    cpu = None
    if not args.no_cpu:
        from oracle import fit as ofit
        import threadpoolctl
        rng = np.random.default_rng(1)
        Lenv = wl.complex_normal(rng, (Dlr, w, Dlr))
        M1, M2 = wl.complex_normal(rng, (Dlr, 2, Dlr)), wl.complex_normal(rng, (Dlr, 2, Dlr))
        t0 = time.perf_counter()
        ofit.env_left(Lenv, M1, W, M1)
        ofit.theta_two_site(Lenv, M1, W, M2, W, Lenv)
        visit = time.perf_counter() - t0
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] + [1])
        cpu = {"value": visit * 4 * (Llr - 1), "unit": "s per time step (extrapolated)", "cores": int(threads),
               "kind": "oracle",
               "sample": f"one bond visit's contractions (one environment update and the projected two-site "
                         f"tensor, D={Dlr}, w={w}) timed in the oracle ({visit:.2f} s, numpy complex128, "
                         f"{threads} BLAS threads), times the {4 * (Llr - 1)} visits of a step; the SVDs "
                         f"are not included"}
    line = {
        "metric": "s per time step & TFLOP/s at D=256: FP32-MFMA grouped vs plain FP64, fidelity",
        "value": sec, "unit": "s per time step", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[args.prec], "data": "synthetic",
        "config": {"workload": f"long-range Ising L={Llr}, J(r)=r^-2 as 6 exponentials, g=1, order-{order} "
                               f"extended MPO (w={w}), tau={tau}, D={Dlr} saturated random MPS",
                   "L": Llr, "D": Dlr, "order": order, "tau": tau},
        "step_gflop": float(np.mean([x.gflop for x in st])),
        "kernel_classes_timed_steps": {
            "jacobi_svd_ms": prof["t_jacobi_ms"], "n_jacobi": prof["n_jacobi"],
            "complex_gemm_ms": prof["t_gemm_ms"], "complex_gemm_gflop": prof["gemm_gflop"],
            "complex_gemm_tflops": gemm_tf, "complex_gemm_frac_of_peak": gemm_tf * 1e12 / peak,
            "w_contraction_ms": prof["t_wmix_ms"]},
        "svd_sweeps_mean": float(np.mean([x.svd_sweeps_total / max(x.visits, 1) for x in st])),
        "fp64_path": fp64,
        "bf16x3_path": bf,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def run_env(args, torch, mp, h):
    """The environment-update microbenchmark alone: FP32 (three real products per complex
    multiply-add on the fp32 matrix cores), plain FP64 and split-BF16x3, K calls each."""
    reps = max(1, args.steps)
    res = {}
    for name in ("fp32", "fp64", "bf16x3"):
        ms, flop = env_microbench(mp, h, torch, prec_of(mp, name), reps=reps)
        peak = 78.6 if name == "fp64" else 157.3
        res[name] = {"us": ms * 1e3, "tflops": flop / ms / 1e9, "frac_of_peak": flop / ms / 1e9 / peak,
                     "peak_tflops": peak}
    f32 = res["fp32"]
    print(json.dumps({
        "metric": "env_update (left) TFLOP/s at D=256, d=2, w=8, FP32 matrix cores",
        "value": f32["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": reps, "warmup": 3,
        "ms_per_step": f32["us"] / 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "left environment update, E (256, 8, 256), ket/bra (256, 2, 256), "
                               "W (8, 2, 2, 8), seeded complex normal operands",
                   "flop_per_call": 8.0 * (2 * 256 ** 3 * 2 * 8 + 256 ** 2 * 2 ** 2 * 8 ** 2)},
        "roofline": {"bound": "mfma", "achieved": f32["tflops"], "peak": 157.3, "unit": "TFLOP/s",
                     "frac": f32["frac_of_peak"], "traffic": None},
        "precisions": res,
    }), flush=True)


def _overlap(a, b) -> complex:
    """<a|b> of two open-boundary MPS given as host arrays (transfer-matrix contraction)."""
    E = np.ones((1, 1), dtype=np.complex128)
    for A, B in zip(a, b):  # pairwise contractions: O(D^3 d) per site
        E = np.tensordot(E, A.conj(), axes=([0], [0]))      # [y, s, u]
        E = np.tensordot(E, B, axes=([0, 1], [0, 1]))       # [u, v]
    return complex(E[0, 0])


def run_split(args, torch, mp, wl, h):
    """K quench steps (default 20) from the g = 0.5 ground state with the splitting composite
    O1(t1 tau) O1(t2 tau) (Sec. 8.3) and with the order-2 MPO, each step timed with HIP events."""
    steps = args.steps if args.steps != 100 else 20
    prec = prec_of(mp, args.prec)
    psi0 = load_ground()
    H = wl.tfim(G_AFTER)
    tau = -1j * TAU
    W2, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, ORDER, tau, mp.V2_EXTENDED)
    Wb, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, 1, mp.SPLIT_T2 * tau, mp.V2_EXTENDED)
    Wa, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, 1, mp.SPLIT_T1 * tau, mp.V2_EXTENDED)
    d2, da, db = mp.DeviceMPO([W2] * L), mp.DeviceMPO([Wa] * L), mp.DeviceMPO([Wb] * L)

    def advance(dm, split, k, ws):
        if split:
            mp.split_step(h, dm, db, da, prec=prec, input_right_canonical=k > 0, workspace=ws)
        else:
            mp.step(h, dm, d2, prec=prec, input_right_canonical=k > 0, workspace=ws)

    def run(split):
        ws = mp.step_workspace(mp.DeviceMPS(psi0, Dmax=D), d2, prec)  # bond 3 covers bond 2
        warm = mp.DeviceMPS(psi0, Dmax=D)
        advance(warm, split, 0, ws)
        torch.cuda.synchronize()
        dm = mp.DeviceMPS(psi0, Dmax=D)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record()
        for k in range(steps):
            advance(dm, split, k, ws)
            ev[k + 1].record()
            if args.progress and k % 10 == 9:
                print(f"[bench] {'split' if split else 'order 2'} step {k + 1}/{steps}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        return [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)], dm

    ms2, dm2 = run(False)
    mss, dms = run(True)
    a, b = dms.to_numpy(), dm2.to_numpy()
    fid = abs(_overlap(a, b)) ** 2 / (abs(_overlap(a, a)) * abs(_overlap(b, b)))
    s_split, s_o2 = float(np.sum(mss)) / 1e3 / steps, float(np.sum(ms2)) / 1e3 / steps
    print(json.dumps({
        "metric": "s per time step, splitting composite O1(t1 tau) O1(t2 tau) vs order-2 MPO",
        "value": s_split, "unit": "s per time step", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": s_split * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPES[args.prec], "data": "synthetic",
        "config": {"workload": f"TFIM quench L={L} from the g=0.5 ground state to g={G_AFTER}, tau={TAU}, "
                               f"D<={D}, 2 sweeps per fit, steps 1..{steps}: splitting composite "
                               f"(first-order MPO, bond 2, at t2 tau then t1 tau) vs the order-2 MPO (bond 3)",
                   "L": L, "D": D, "tau": TAU},
        "order2_s_per_step": s_o2,
        "split_over_order2": s_split / s_o2,
        "trajectory_infidelity": 1.0 - fid,
        "max_bond_split": max(dms.bond), "max_bond_order2": max(dm2.bond),
    }), flush=True)


def run_thermal(args, torch, mp, wl, h):
    """Imaginary-time steps of the purified L = 64 TFIM (g = 1) from beta = 0, FP32 and FP64."""
    steps = args.steps if args.steps != 100 else 20
    delta, g = 0.05, 1.0
    H = wl.tfim(g)
    W, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, ORDER, -delta, mp.V2_EXTENDED)
    dw = mp.DeviceMPO([mp.purify_mpo(W)] * L)
    Hm = np.zeros((3, 2, 2, 3), dtype=np.complex128)
    Hm[0, :, :, 0] = Hm[2, :, :, 2] = np.eye(2)
    Hm[0, :, :, 1], Hm[1, :, :, 2], Hm[0, :, :, 2] = H.C[0], H.B[0], H.Dloc
    dH = mp.DeviceMPO([mp.purify_mpo(Hm)] * L)
    psi0 = wl.infinite_temperature(L)

    def run(prec):
        ws = mp.step_workspace(mp.DeviceMPS(psi0, Dmax=D), dw, prec)
        warm = mp.DeviceMPS(psi0, Dmax=D)
        mp.step(h, warm, dw, prec=prec, workspace=ws)
        torch.cuda.synchronize()
        dm = mp.DeviceMPS(psi0, Dmax=D)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record()
        for k in range(steps):
            mp.step(h, dm, dw, prec=prec, input_right_canonical=k > 0, workspace=ws)
            ev[k + 1].record()
            if args.progress and k % 10 == 9:
                print(f"[bench] thermal prec {prec} step {k + 1}/{steps}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
        return float(np.sum(ms)) / 1e3 / steps, mp.expectation(h, dm, dH, 0, 2).real / L, max(dm.bond)

    s32, e32, b32 = run(mp.FP32)
    s64, e64, b64 = run(mp.FP64)
    print(json.dumps({
        "metric": "s per imaginary-time step, purified TFIM (finite temperature)",
        "value": s32, "unit": "s per time step", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": s32 * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPES["fp32"], "data": "synthetic",
        "config": {"workload": f"TFIM L={L}, g={g}, purified (d=4), order-{ORDER} extended MPO at tau=-{delta} "
                               f"on the physical legs, D<={D}, beta 0 -> {2 * delta * steps:g}",
                   "L": L, "D": D, "order": ORDER, "delta": delta},
        "beta_end": 2 * delta * steps,
        "energy_per_site_fp32": e32, "energy_per_site_fp64": e64,
        "fp64_s_per_step": s64, "fp32_speedup": s64 / s32,
        "max_bond_fp32": b32, "max_bond_fp64": b64,
    }), flush=True)


def run_cylinder(args, torch, mp, wl, h):
    """Fidelity density after T = 1 against the time step for orders 1-3 on a W = 4 cylinder."""
    Ly, Lx, hx, Dc, T = 4, 8, 2.0, 64, 1.0
    N = Ly * Lx
    prec = prec_of(mp, args.prec)
    H = wl.tfim_cylinder(Ly, hx)

    def evolve(psi, order, tau, steps, canonical=False):
        W, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, order, tau, mp.V2_EXTENDED)
        dw = mp.DeviceMPO([W] * N)
        dm = mp.DeviceMPS(psi, Dmax=Dc)
        ws = mp.step_workspace(dm, dw, prec)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record()
        for k in range(steps):
            mp.step(h, dm, dw, prec=prec, input_right_canonical=canonical or k > 0, workspace=ws)
            ev[k + 1].record()
        torch.cuda.synchronize()
        return dm.to_numpy(), float(sum(ev[k].elapsed_time(ev[k + 1]) for k in range(steps))) / 1e3

    # ground state: imaginary-time steps of the order-2 MPO from all-up (beta / 2 = 6)
    gs, t_gs = evolve(wl.all_up(N), 2, -0.1, 60)
    if args.progress:
        print(f"[bench] cylinder ground state {t_gs:.1f} s", file=sys.stderr, flush=True)
    flipped = [m.copy() for m in gs]
    mid = N // 2
    flipped[mid] = np.einsum('st,atb->asb', wl.SX, flipped[mid])

    def unit(ms):
        n = np.sqrt(abs(_overlap(ms, ms)))
        out = [m.copy() for m in ms]
        out[0] = out[0] / n
        return out

    ref, t_ref = evolve(flipped, 3, -1j * 0.0125, 80)
    ref = unit(ref)
    rows = []
    for order in (1, 2, 3):
        for dt in (0.2, 0.1, 0.05):
            steps = int(round(T / dt))
            out, t = evolve(flipped, order, -1j * dt, steps)
            f = float(np.log(abs(_overlap(ref, unit(out))))) / N
            rows.append({"order": order, "dt": dt, "steps": steps, "fidelity_density": f,
                         "gpu_s": t, "s_per_step": t / steps})
            if args.progress:
                print(f"[bench] cylinder order {order} dt {dt}: f = {f:.3e}, {t:.2f} s", file=sys.stderr, flush=True)
    o2 = [r for r in rows if r["order"] == 2 and r["dt"] == 0.1][0]
    print(json.dumps({
        "metric": "fidelity density after T=1 vs time step, orders 1-3, W=4 spiral cylinder",
        "value": o2["s_per_step"], "unit": "s per time step (order 2, dt = 0.1)", "n_gpus": 1,
        "steps": o2["steps"], "warmup": 0, "ms_per_step": o2["s_per_step"] * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": DTYPES[args.prec],
        "data": "synthetic",
        "config": {"workload": f"TFIM on a W={Ly} spiral cylinder, {Lx}x{Ly}={N} sites, h={hx}, D<={Dc}, "
                               "ground state by 60 imaginary-time steps (order 2, tau=-0.1), spin flip "
                               "(X) on the middle site, evolution to T=1; reference: order 3, dt=0.0125",
                   "Ly": Ly, "Lx": Lx, "h": hx, "D": Dc, "T": T},
        "reference_gpu_s": t_ref, "ground_state_gpu_s": t_gs,
        "runs": rows,
    }), flush=True)


def run_batched(args, torch, mp, wl, h):
    """K steps of 64 independent TFIM chains (g ~ U(0.5, 1.5), L in {32, 64, 96, 128}, D in
    {32, 64, 128, 256}, seed 2), order-2 extended MPO, tau = 0.1, from all-up: step_batched
    against the same chains stepped one by one, and the oracle on the first chains' first step."""
    chains = wl.batched_tfim_chains(2, 64)
    steps = args.steps if args.steps != 100 else 3
    prec = prec_of(mp, args.prec)
    mpos = {}
    for g, Lc, _ in chains:
        if g not in mpos:
            H = wl.tfim(g)
            mpos[g] = mp.mpo_build(H.A, H.B, H.C, H.Dloc, 2, -1j * TAU, mp.V2_EXTENDED)[0]
    dws = [mp.DeviceMPO([mpos[g]] * Lc) for g, Lc, _ in chains]

    def trajectory(batched):
        dms = [mp.DeviceMPS(wl.all_up(Lc), Dmax=Dc) for _, Lc, Dc in chains]
        if batched:
            ws = mp.step_batched_workspace(dms, dws, prec)
        else:
            ws = [mp.step_workspace(dm, dw, prec) for dm, dw in zip(dms, dws)]
        torch.cuda.synchronize()
        ms, first = [], None
        for k in range(steps):
            t0 = time.perf_counter()
            if batched:
                st = mp.step_batched(h, dms, dws, prec=prec, workspace=ws, input_right_canonical=k > 0)
            else:
                st = [mp.step(h, dm, dw, prec=prec, workspace=w_, input_right_canonical=k > 0)
                      for dm, dw, w_ in zip(dms, dws, ws)]
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
            if k == 0:
                first = [dm.to_numpy() for dm in dms[:4]]
        bonds = [max(dm.bond) for dm in dms]
        gflop = sum(x.gflop for x in st)
        del ws, dms
        torch.cuda.empty_cache()
        return ms, first, bonds, gflop

    ms_b, first_b, bonds, gflop = trajectory(True)
    ms_1, first_1, _, _ = trajectory(False)
    sec = float(np.sum(ms_b)) / 1e3 / steps
    parity, cpu = None, None
    if not args.no_cpu:
        from oracle import fit as ofit
        import threadpoolctl
        parity = []
        t0 = time.perf_counter()
        for c in range(4):
            g, Lc, Dc = chains[c]
            ref, _ = ofit.fit_step(wl.all_up(Lc), mpos[g], Dmax=Dc, nsweeps=2)
            parity.append({"chain": c, "L": Lc, "D": Dc, "g": g,
                           "step1_infidelity": float(1.0 - abs(ofit.overlap(first_b[c], ref)) ** 2),
                           "batched_vs_one_by_one_max_abs": float(max(np.max(np.abs(a - b)) for a, b in
                                                                      zip(first_b[c], first_1[c])))})
        cpu_s = time.perf_counter() - t0
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] + [1])
        cpu = {"value": cpu_s, "unit": "s for step 1 of chains 0-3", "cores": int(threads), "kind": "oracle",
               "sample": f"the oracle's first step (from all-up) of the first four chains, numpy complex128 with "
                         f"{threads} BLAS threads; the GPU batch takes steps_ms[0] for all 64 chains"}
    line = {
        "metric": "s per time step & TFLOP/s at D=256: FP32-MFMA grouped vs plain FP64, fidelity",
        "value": sec, "unit": "s per time step (64 chains)", "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": sec * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[args.prec], "data": "synthetic",
        "config": {"workload": "64 independent TFIM chains, g ~ U(0.5,1.5), L in {32,64,96,128}, "
                               "D in {32,64,128,256} (seed 2), order-2 extended MPO (w=3), tau=0.1, "
                               f"2 sweeps, all-up start, steps 1..{steps}",
                   "chains": len(chains), "tau": TAU, "order": 2},
        "steps_ms_batched": ms_b, "steps_ms_one_by_one": ms_1,
        "batched_speedup": float(np.sum(ms_1) / np.sum(ms_b)),
        "chain_steps_per_s": len(chains) * steps / (float(np.sum(ms_b)) / 1e3),
        "worker_streams_requested": int(os.environ.get("MPOEVO_BATCH_STREAMS", "4")),
        "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"),
        "last_step_gflop": gflop, "max_bond_per_chain_end": bonds,
        "parity_vs_oracle": parity,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def main():
    global ORDER, TAU
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", choices=["fp32", "fp64", "bf16x3"], default="fp32")
    ap.add_argument("--fp64-steps", type=int, default=20, help="opening steps run on the FP64 path too")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and parity")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--workload", choices=["quench", "lr3", "batched", "env", "split", "thermal", "cylinder"], default="quench")
    ap.add_argument("--progress", action="store_true", help="print a line to stderr every 10 timed steps")
    ap.add_argument("--order", type=int, default=ORDER, choices=[1, 2, 3, 4],
                    help="MPO order of the TFIM workloads (quench, split reference, thermal)")
    ap.add_argument("--tau", type=float, default=TAU, help="time step of the quench and split workloads")
    args = ap.parse_args()
    ORDER, TAU = args.order, args.tau
    if args.workload == "batched":
        # more hardware queues and worker streams let more chains' truncations overlap (read by
        # the HIP runtime at initialisation and by the library at each batched step)
        os.environ.setdefault("GPU_MAX_HW_QUEUES", "8")
        os.environ.setdefault("MPOEVO_BATCH_STREAMS", "8")
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the time step of a single chain is sequential across "
              "bonds and this build has no multi-GPU path (the design notes describe how it would "
              "shard).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2302_14181_amd import mpoevo as mp
    from paper_2302_14181_amd import workloads as wl

    torch.cuda.set_device(0)
    h = mp.Handle(0)
    if args.workload == "env":
        run_env(args, torch, mp, h)
        h.close()
        return
    if args.workload in ("split", "thermal", "cylinder"):
        {"split": run_split, "thermal": run_thermal, "cylinder": run_cylinder}[args.workload](args, torch, mp, wl, h)
        h.close()
        return
    if args.workload in ("lr3", "batched"):
        (run_lr3 if args.workload == "lr3" else run_batched)(args, torch, mp, wl, h)
        h.close()
        return
    prec = prec_of(mp, args.prec)
    psi0 = load_ground()
    H = wl.tfim(G_AFTER)
    W, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, ORDER, -1j * TAU, mp.V2_EXTENDED)
    dw = mp.DeviceMPO([W] * L)

    def quench(p, steps, warmup, profile=False):
        """Per-step milliseconds of `steps` quench steps from psi0 (events on the default stream);
        with `profile` every step also times its kernel classes with HIP events."""
        if warmup:
            dm = mp.DeviceMPS(psi0, Dmax=D)
            wsw = mp.step_workspace(dm, dw, p)
            for k in range(warmup):
                mp.step(h, dm, dw, prec=p, input_right_canonical=k > 0, workspace=wsw)
            torch.cuda.synchronize()
            del wsw
        dm = mp.DeviceMPS(psi0, Dmax=D)
        ws = torch.empty_like(mp.step_workspace(dm, dw, p))
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        st = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record()
        for k in range(steps):
            st.append(mp.step(h, dm, dw, prec=p, input_right_canonical=k > 0, workspace=ws,
                              profile=profile))
            ev[k + 1].record()
            if args.progress and k % 10 == 9:
                print(f"[bench] step {k + 1}/{steps}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
        return ms, wall, st, dm

    # the timed steps time the Jacobi kernel only (HIP events around each launch, on its stream):
    # events around every kernel class would add a few per cent of host work to the steps
    ms, wall, st, dm_end = quench(prec, args.steps, args.warmup, profile=mp.PROFILE_JACOBI)
    sec_step = float(np.sum(ms)) / 1e3 / args.steps
    gflop = float(np.mean([x.gflop for x in st]))

    def class_table(prof):
        classes = {
            "jacobi_svd": {"ms": prof["t_jacobi_ms"], "launches": prof["n_jacobi"], "work": prof["jacobi_gflop"],
                           "work_unit": "GFLOP", "bound": "alu", "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s"},
            "complex_gemm": {"ms": prof["t_gemm_ms"], "launches": prof["n_gemm"], "work": prof["gemm_gflop"],
                             "work_unit": "GFLOP", "bound": "mfma",
                             "peak": {mp.FP32: PEAK_FP32_MFMA, mp.FP64: PEAK_FP64_MFMA,
                                      mp.BF16X3: CEIL_BF16X3}[prec] / 1e12, "unit": "TFLOP/s"},
            "w_contraction": {"ms": prof["t_wmix_ms"], "launches": prof["n_wmix"], "work": prof["wmix_gbyte"],
                              "work_unit": "GB", "bound": "hbm", "peak": PEAK_HBM / 1e9, "unit": "GB/s"},
        }
        for c in classes.values():
            c["achieved"] = c["work"] / (c["ms"] * 1e-3) / (1e3 if c["unit"] == "TFLOP/s" else 1.0) if c["ms"] > 0 else 0.0
            c["frac"] = c["achieved"] / c["peak"] if c["peak"] else 0.0
            c["avg_launch_us"] = 1e3 * c["ms"] / max(c["launches"], 1)
        return classes

    # the Jacobi kernel summed over the timed steps (the dominant kernel: the roofline below)
    prof = {k: float(sum(x.profile[k] for x in st)) for k in st[0].profile}
    classes = {"jacobi_svd": class_table(prof)["jacobi_svd"]}
    dominant = "jacobi_svd"

    # diagnostics of the trajectory on the device (FP64): energy of H(g = 1.5), conserved by the
    # exact evolution, and <Z_32>, at t = 0 and after the last timed step
    Hm = np.zeros((3, 2, 2, 3), dtype=np.complex128)
    Hm[0, :, :, 0] = Hm[2, :, :, 2] = np.eye(2)
    Hm[0, :, :, 1], Hm[1, :, :, 2], Hm[0, :, :, 2] = H.C[0], H.B[0], H.Dloc
    dH = mp.DeviceMPO([Hm] * L)
    Id = np.eye(2, dtype=np.complex128).reshape(1, 2, 2, 1)
    zops = [Id] * L
    zops[31] = wl.SZ.reshape(1, 2, 2, 1)
    dZ = mp.DeviceMPO(zops)
    dm0 = mp.DeviceMPS(psi0, Dmax=D)
    diag = {"energy_t0": mp.expectation(h, dm0, dH, 0, 2).real,
            "energy_end": mp.expectation(h, dm_end, dH, 0, 2).real,
            "Z32_t0": mp.expectation(h, dm0, dZ).real,
            "Z32_end": mp.expectation(h, dm_end, dZ).real,
            "t_end": TAU * args.steps}
    diag["energy_drift_per_site"] = (diag["energy_end"] - diag["energy_t0"]) / L
    del dm0, dm_end

    # the plain FP64 path on the same opening steps
    fp64 = None
    if not args.no_fp64 and prec == mp.FP32:
        n64 = max(1, min(args.fp64_steps, args.steps))
        ms64, _, _, dm64 = quench(mp.FP64, n64, 0, profile=True)
        fp64 = {"steps": n64, "fp64_s_per_step": float(np.sum(ms64)) / 1e3 / n64,
                "fp32_s_per_step": float(np.sum(ms[:n64])) / 1e3 / n64}
        fp64["fp32_speedup"] = fp64["fp64_s_per_step"] / fp64["fp32_s_per_step"]
        # the FP32 and FP64 trajectories after the same n64 steps from psi0
        _, _, _, dm32n = quench(mp.FP32, n64, 0)
        a, b = dm32n.to_numpy(), dm64.to_numpy()
        fp64["trajectory_infidelity_fp32_vs_fp64"] = 1.0 - abs(_overlap(a, b)) ** 2 / (
            abs(_overlap(a, a)) * abs(_overlap(b, b)))
        fp64["Z32_after_steps_fp32"] = mp.expectation(h, dm32n, dZ).real
        fp64["Z32_after_steps_fp64"] = mp.expectation(h, dm64, dZ).real

    # one step at saturated bond dimension (seeded random MPS, D = 128 on every bulk bond), after
    # two steps that leave the truncations' preconditioners in the workspace
    # (a fourth step, timing every kernel class, gives the breakdown of a saturated step)
    rnd = wl.random_mps(np.random.default_rng(0), L, 2, D)

    def saturated_step(p, breakdown=False):
        dmr = mp.DeviceMPS(rnd, Dmax=D)
        wsr = mp.step_workspace(dmr, dw, p)
        mp.step(h, dmr, dw, prec=p, workspace=wsr)
        mp.step(h, dmr, dw, prec=p, input_right_canonical=True, workspace=wsr)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        mp.step(h, dmr, dw, prec=p, input_right_canonical=True, workspace=wsr)
        e.record()
        torch.cuda.synchronize()
        t = s.elapsed_time(e) / 1e3
        if not breakdown:
            return t, None
        sp = mp.step(h, dmr, dw, prec=p, input_right_canonical=True, workspace=wsr, profile=True)
        torch.cuda.synchronize()
        return t, class_table(sp.profile)

    sat_s, sat_classes = saturated_step(prec, breakdown=True)
    if fp64 is not None:  # the same saturated step on the plain FP64 path
        fp64["saturated_fp64_s_per_step"] = saturated_step(mp.FP64)[0]
        fp64["saturated_fp32_s_per_step"] = sat_s
        fp64["saturated_fp32_speedup"] = fp64["saturated_fp64_s_per_step"] / sat_s

    mb32_ms, mb_flop = env_microbench(mp, h, torch, mp.FP32)
    mb64_ms, _ = env_microbench(mp, h, torch, mp.FP64)
    mbbf_ms, _ = env_microbench(mp, h, torch, mp.BF16X3)
    d256 = None if args.no_fp64 else run_lr3(args, torch, mp, wl, h, steps=1, warmup=1, embedded=True)

    # parity of the first step from psi0 against the oracle, and the CPU baseline
    cpu = None
    parity = None
    if not args.no_cpu:
        from oracle import fit as ofit
        import threadpoolctl
        ref, rinfo = ofit.fit_step(psi0, W, Dmax=D, nsweeps=2)
        parity = {}
        for name, p in (("fp32", mp.FP32), ("fp64", mp.FP64), ("bf16x3", mp.BF16X3)):
            dm1 = mp.DeviceMPS(psi0, Dmax=D)
            s1 = mp.step(h, dm1, dw, prec=p)
            out = dm1.to_numpy()
            parity[name] = {
                "step1_infidelity": float(1.0 - abs(ofit.overlap(out, ref)) ** 2),
                "step1_Z32_error": float(abs(ofit.expect_local(out, wl.SZ, 31) - ofit.expect_local(ref, wl.SZ, 31))),
                "step1_norm_rel_error": float(abs(s1.norm - rinfo["norm"]) / rinfo["norm"]),
            }
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] + [1])
        t0 = time.perf_counter()
        ofit.fit_step(rnd, W, Dmax=D, nsweeps=2)
        cpu_s = time.perf_counter() - t0
        cpu = {"value": cpu_s, "unit": "s per time step", "cores": int(threads), "kind": "oracle",
               "sample": f"one time step at saturated bond dimension (seeded random MPS, L={L}, D={D} on "
                         f"every bulk bond, order {ORDER}, 2 sweeps, including its right-canonicalisation), "
                         f"numpy complex128 with {threads} BLAS threads on {os.cpu_count()} host cores; "
                         f"the GPU takes gpu_saturated_step_s for the same step",
               "gpu_saturated_step_s": sat_s}

    mb_tflops = mb_flop / (mb32_ms * 1e-3) / 1e12
    phases = {}
    for lo, hi in ((0, 20), (20, 40), (40, args.steps)):
        if hi > lo and lo < args.steps:
            seg = ms[lo:min(hi, args.steps)]
            phases[f"steps_{lo + 1}_{min(hi, args.steps)}_ms"] = float(np.mean(seg))
    line = {
        "metric": "s per time step & TFLOP/s at D=256: FP32-MFMA grouped vs plain FP64, fidelity",
        "value": sec_step,
        "unit": "s per time step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_step * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.prec],
        "data": "synthetic",
        "config": {"workload": f"TFIM quench L={L} from the g=0.5 ground state to g={G_AFTER}, order-{ORDER} "
                               f"extended MPO (w={W.shape[0]}), tau={TAU}, D<={D}, 2 sweeps per step, "
                               f"steps 1..{args.steps} from t=0",
                   "L": L, "D": D, "order": ORDER, "tau": TAU},
        "wall_s_per_step": wall / args.steps,
        "phase_ms_per_step": phases,
        "max_bond_last_step": int(st[-1].max_bond),
        "discarded_sum_last_step": float(st[-1].discarded_sum),
        "step_gflop_mean": gflop,
        "svd_sweeps_mean": float(np.mean([x.svd_sweeps_total / max(x.visits, 1) for x in st])),
        "fp64_path": fp64,
        "diagnostics_device": diag,
        "gpu_saturated_step_s": sat_s,
        "parity_vs_oracle": parity,
        "d256_long_range": d256,
        "env_microbench": {"D": 256, "d": 2, "w": 8, "fp32_ms": mb32_ms, "fp64_ms": mb64_ms,
                           "fp32_tflops": mb_tflops, "fp64_tflops": mb_flop / (mb64_ms * 1e-3) / 1e12,
                           "fp32_frac_of_mfma_peak": mb_tflops * 1e12 / PEAK_FP32_MFMA,
                           "fp64_frac_of_mfma_peak": mb_flop / (mb64_ms * 1e-3) / PEAK_FP64_MFMA,
                           "bf16x3_ms": mbbf_ms, "bf16x3_tflops": mb_flop / (mbbf_ms * 1e-3) / 1e12,
                           "bf16x3_frac_of_ceiling": mb_flop / (mbbf_ms * 1e-3) / CEIL_BF16X3},
        "roofline": {"bound": classes[dominant]["bound"], "kernel": dominant,
                     "achieved": classes[dominant]["achieved"], "peak": classes[dominant]["peak"],
                     "unit": classes[dominant]["unit"], "frac": classes[dominant]["frac"],
                     "avg_launch_us": classes[dominant]["avg_launch_us"], "traffic": None},
        "kernel_classes_timed_steps": classes,
        "kernel_classes_saturated_step": sat_classes,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    h.close()


if __name__ == "__main__":
    main()
