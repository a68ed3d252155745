"""Benchmark: seconds per time step of the variational higher-order MPO evolution on one MI355X.

Workload (default, --workload lr3): the long-range Ising chain H = -sum_{i<j} J(j-i) Z_i Z_j - g sum X_i
with J(r) = r^-2 fitted as six exponentials (tests/golden/lr_fit_K6.json), g = 1, L = 100, the
order-3 extended MPO (w = 271) of exp(-i tau H), tau = 0.1, bond dimension D <= 256, cutoff
1e-14 sigma_1, two sweeps per step (two-site updates while the bonds grow, one-site updates at the
bonds already at their largest value; --nsites), from the all-up product state: K time steps from
t = 0 (default K = 20) after W untimed warm-up steps of the same trajectory on their own state
(default W = 2). Contractions on the FP32 matrix cores (--prec), the SVD truncation and the QR in
FP64. The bonds reach D = 256 at step 3. A step whose plan the handle has seen before (the warm-up
steps are the first sightings) is captured into a HIP graph and replayed (--no-graph: kernel by
kernel); the kernel table comes from the same K steps run again launch by launch. `value` is the
mean seconds per step over the K timed steps (HIP events on the launch stream around each step;
every step ends with a synchronisation).

Also on the line: the plain FP64 path (kernel by kernel) on the same K opening steps (time ratio, and the two
trajectories' infidelity and <Z_50> after them); per-step parity against the CPU oracle on the
opening steps: step 1 from all-up on every precision (R17-A infidelity 1 - |<phi_gpu|phi_oracle>|^2
and R17-B |eps_gpu - eps_oracle|, eps = 1 - |<phi|W psi>|^2 / ||W psi||^2) and step 2 restarted from
the oracle's state after step 1; the timed launches of the K steps per kernel instance with their
algorithmic rates, the dominant one as the roofline line (with the HBM traffic per launch from
profiles/hbm_traffic_lr3.md while the measured source is unchanged); the CPU oracle timed on
saturated bond visits and scaled to a step (cpu_baseline); side fields: the L = 64 TFIM quench
(configuration 2, steps 1-20, FP32 and FP64, first-step parity) and the environment-update
microbenchmark at D = 256, d = 2, w = 8.

--workload quench: the L = 64 TFIM quench g = 0.5 -> 1.5 from the ground state at g = 0.5
(tests/golden/tfim_g05_L64_ground.npz, prepared by the oracle), order-2 extended MPO (w = 3; --order),
tau = 0.1 (--tau), D <= 128, K steps (default 100) with the FP64 comparison and first-step parity.

--workload xxz: the XXZ chain with U(1) charges (configuration 4): L = 128, 64 up spins, Delta = 0.5,
order-2 extended MPO (w = 13), tau = 0.1, D <= 512 over about 15 charge sectors per bond (seeded
sector tables), K steps (default 20) from a seeded random U(1) state, FP32 and FP64, parity of step 1
against the block-sparse oracle.

--workload batched: 64 independent TFIM chains (g ~ U(0.5, 1.5), L in {32, 64, 96, 128},
D in {32, 64, 128, 256}, seed 2), order-2 extended MPO, tau = 0.1, from all-up, K steps (default 3)
advanced together by step_batched, against the same steps taken chain by chain; the oracle checks
and times the first step of the first four chains.

--workload split: the quench advanced by the splitting composite of Sec. 8.3 (the first-order MPO at
t2 tau, then at t1 tau, t1,2 = (1 +- i)/2: two fits per step at MPO bond 2) against the order-2 MPO
(one fit at bond 3), K steps each (default 20) from the same state.

--workload thermal: finite temperature by purification on the L = 64 TFIM at g = 1 (physical and
ancilla leg per site, d = 4): the order-2 MPO at tau = -0.05 on the physical legs, K steps (default
20) from beta = 0 to beta = 2 K 0.05, D <= 128; FP32 and FP64 paths.

--workload cylinder: the efficiency set-up of Sec. 8.2 on a finite W = 4 spiral cylinder (TFIM, h = 2,
8 x 4 = 32 sites, D <= 64): fidelity density after T = 1 against the time step for orders 1-3
against an order-3 run at dt = 0.0125 (standing in for the TDVP reference).

--workload env: only the left environment update at D = 256, d = 2, w = 8, K calls per precision
(default 100) timed with HIP events on the launch stream; --env-w 271: the same at the long-range
chain's MPO (w = 271, default 10 calls), whose products are the default line's dominant kernel.

--workload copy: a plain 256 MiB device copy, K times (the calibration of the HBM counters).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec fp32|fp64|bf16x3] [--fp64-steps N]
                       [--no-cpu] [--no-fp64] [--no-delta2] [--no-side] [--nsites -1|1|2]
                       [--guess canonical|zipup|auto] [--graph] [--no-graph] [--tune] [--env-w 8|271]
                       [--workload lr3|quench|xxz|batched|env|split|thermal|cylinder|copy]
                       [--order N] [--tau T] [--quiet]
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


def env_inputs(mp, wl, w: int):
    """Operands of the environment microbenchmark: w = 8, the seeded complex-normal set of
    workloads.env_microbench_inputs; w = 271, the long-range chain's order-3 MPO with E, ket and
    bra (256, 271, 256), (256, 2, 256) x 2 complex normal from default_rng(0) in that order."""
    if w == 8:
        return wl.env_microbench_inputs(0)
    H = lr_blocks(wl)
    W, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, LR_ORDER, -1j * LR_TAU, mp.V2_EXTENDED)
    if W.shape[0] != w:
        raise SystemExit(f"--env-w {w}: the long-range MPO has w = {W.shape[0]}")
    rng = np.random.default_rng(0)
    E = wl.complex_normal(rng, (256, w, 256))
    M = wl.complex_normal(rng, (256, 2, 256))
    N = wl.complex_normal(rng, (256, 2, 256))
    return E, M, N, W


def env_warmup(w: int) -> int:
    """Untimed env_update calls before the timed ones (tens of ms of work: the device at its
    steady clock)."""
    return 100 if w == 8 else 10


def env_microbench(mp, h, torch, prec: int, reps: int = 200, w: int = 8):
    """Time env_update (left) at D = 256, d = 2 and MPO bond w with HIP events on the launch stream,
    after env_warmup(w) untimed calls, averaged over `reps` calls."""
    from paper_2302_14181_amd import workloads as wl
    E, M, N, W = env_inputs(mp, wl, w)
    dt = torch.complex128 if prec == mp.FP64 else torch.complex64
    t = {k: torch.from_numpy(v).to(dt).cuda() for k, v in dict(E=E, M=M, N=N, W=W).items()}
    del E, M, N
    out = torch.empty((256, w, 256), dtype=dt, device="cuda")
    ws = torch.empty(mp.workspace_size(mp.CALL_ENV_UPDATE, [256, 256, 256, 256, 2, w, w], prec),
                     dtype=torch.uint8, device="cuda")
    for _ in range(env_warmup(w)):
        mp.env_update(h, mp.LEFT, t["E"], t["N"], t["W"], t["M"], out, workspace=ws, prec=prec)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        mp.env_update(h, mp.LEFT, t["E"], t["N"], t["W"], t["M"], out, workspace=ws, prec=prec)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    Dm, d = 256, 2
    flop = 8.0 * (2 * Dm ** 3 * d * w + Dm ** 2 * d ** 2 * w ** 2)
    del t, out, ws
    torch.cuda.empty_cache()
    return ms, flop


def load_ground():
    z = np.load(GROUND)
    return [z[f"site_{i:03d}"] for i in range(L)]


LR_L, LR_D, LR_ORDER, LR_TAU, LR_SITE = 100, 256, 3, 0.1, 49  # <Z> on site 50 (counted from 1)
NSITES_DESC = {2: "two-site updates", 1: "one-site updates at fixed bonds",
               -1: "two-site updates while the bonds grow, one-site once every bond is at its largest value"}


def lr_blocks(wl):
    """J(r) = r^-2 as six exponentials (tests/golden/lr_fit_K6.json), transverse field g = 1."""
    fit = json.load(open(os.path.join(ROOT, "tests", "golden", "lr_fit_K6.json")))
    return wl.lr_ising(np.array(fit["coeffs"]), np.array(fit["lambdas"]), 1.0)


GUESS_DESC = {"canonical": "", "zipup": ", each step from the zip-up of W psi",
              "auto": ", from the zip-up of W psi while the bonds grow"}


def guess_of(mp, args):
    return {"canonical": mp.GUESS_CANONICAL, "zipup": mp.GUESS_ZIPUP, "auto": mp.GUESS_AUTO}[args.guess]


def update_kind(st):
    """The updates a step took: one-site, two-site or mixed (with its count of one-site visits)."""
    if st.one_site_visits == st.visits:
        return "one-site"
    if st.one_site_visits == 0:
        return "two-site" + (" (redone)" if st.two_site_redo else "")
    return f"mixed, {st.one_site_visits}/{st.visits} one-site"


def trajectory(torch, mp, h, psi0, dw, prec, steps, Dmax, profile=False, progress=None, nsites=2, guess=0,
               use_graph=False):
    """`steps` time steps from psi0 on a fresh MPS and workspace; HIP events on the launch stream
    around every step. Returns (ms per step, StepStats per step, the final DeviceMPS)."""
    dm = mp.DeviceMPS(psi0, Dmax=Dmax)
    ws = mp.step_workspace(dm, dw, prec)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    st = []
    torch.cuda.synchronize()
    ev[0].record()
    for k in range(steps):
        st.append(mp.step(h, dm, dw, prec=prec, input_right_canonical=k > 0, workspace=ws, profile=profile,
                          nsites=nsites, guess=guess, use_graph=use_graph))
        ev[k + 1].record()
        if progress:
            print(f"[bench] {progress} step {k + 1}/{steps}: bond {st[-1].max_bond}, "
                  f"{update_kind(st[-1])}"
                  f"{', zip-up guess' if st[-1].guess else ''}{', graph' if st[-1].graph else ''}",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    del ws
    torch.cuda.empty_cache()
    return ms, st, dm


PEAKS = {  # by kernel class and contraction precision: (bound, peak, unit)
    ("jacobi_svd", None): ("alu", PEAK_FP64_VALU / 1e12, "TFLOP/s"),
    ("complex_gemm", "fp32"): ("mfma", PEAK_FP32_MFMA / 1e12, "TFLOP/s"),
    ("complex_gemm", "fp64"): ("mfma", PEAK_FP64_MFMA / 1e12, "TFLOP/s"),
    ("complex_gemm", "bf16x3"): ("mfma", PEAK_BF16_MFMA / 1e12, "TFLOP/s"),
    ("w_contraction", None): ("hbm", PEAK_HBM / 1e9, "GB/s"),
    ("householder_qr", None): ("alu", PEAK_FP64_VALU / 1e12, "TFLOP/s"),
}


def kernel_table(stats, prec_name):
    """The profiled launches of a set of steps grouped by kernel instance, longest first, each
    with its algorithmic rate against its roofline (products: 8 flop per complex multiply-add;
    the three-product FP32 kernel issues 6 of them on the matrix cores: `executed_frac`)."""
    agg = {}
    for s in stats:
        for k in s.profile["kernels"]:
            a = agg.setdefault((k["name"], k["split_k"]), {"name": k["name"], "kind": k["kind"],
                                                           "split_k": k["split_k"], "launches": 0,
                                                           "ms": 0.0, "work": 0.0})
            a["launches"] += k["launches"]
            a["ms"] += k["ms"]
            a["work"] += k["work"]
    rows = sorted(agg.values(), key=lambda r: -r["ms"])
    for r in rows:
        bound, peak, unit = PEAKS[(r["kind"], prec_name if r["kind"] == "complex_gemm" else None)]
        scale = 1e3 if unit == "TFLOP/s" else 1.0  # work in GFLOP or GB
        r["avg_launch_us"] = 1e3 * r["ms"] / max(r["launches"], 1)
        r["work_per_launch"] = r["work"] / max(r["launches"], 1)
        r["work_unit"] = "GFLOP" if unit == "TFLOP/s" else "GB"
        r["achieved"] = r["work"] / (r["ms"] * 1e-3) / scale if r["ms"] > 0 else 0.0
        r.update(bound=bound, peak=peak, unit=unit, frac=r["achieved"] / peak)
        if "cgemm3m_kernel" in r["name"]:
            r["executed_frac"] = 0.75 * r["frac"]
    return rows


def roofline_of(row):
    out = {"bound": row["bound"], "kernel": row["name"], "achieved": row["achieved"], "peak": row["peak"],
           "unit": row["unit"], "frac": row["frac"], "avg_launch_us": row["avg_launch_us"],
           "work_per_launch": row["work_per_launch"], "work_unit": row["work_unit"],
           "launches": row["launches"], "traffic": traffic_of(row["name"])}
    if "executed_frac" in row:
        out["executed_frac"] = row["executed_frac"]
    return out


def traffic_of(kernel_name):
    """HBM bytes per launch of a kernel instance from the committed counter summary
    (profiles/hbm_traffic_lr3.md: FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel factors),
    valid only while the source file it was measured on is unchanged; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_lr3.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if not line.startswith("| traffic |"):
            continue
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        _, name, src, sha, fetch, write = cells[:6]
        if name != kernel_name:
            continue
        cur = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()[:16]
        if cur != sha:
            return None
        return float(fetch) + float(write)
    return None


def lr3_parity(torch, mp, h, wl, W, Wo, dw, psi0, Dmax, delta2=True, nsites=-1):
    """Per-step parity against the oracle on the opening steps of the trajectory from all-up:
    step 1 from psi0 (R17-A: 1 - |<phi_gpu|phi_oracle>|^2; R17-B: |eps_gpu - eps_oracle| with
    eps = 1 - |<phi|W psi>|^2 / ||W psi||^2, the device state's overlap with W psi0 taken in FP64 on
    the device, ||W psi0||^2 from the oracle's double-layer contraction) on every contraction precision, and step 2 restarted from the oracle's state
    after step 1 (delta_2, R17-A; the norm error in place of R17-B, whose ||W psi1||^2 is beyond the
    oracle's budget) with the trajectory's update mode: from the oracle's step-1 state the edge
    bonds are already at their largest values, so the automatic mode runs a mixed sweep there,
    against the oracle's fit_step_mixed."""
    from oracle import fit as ofit
    t0 = time.perf_counter()
    ref1, r1 = ofit.fit_step(psi0, Wo, Dmax=Dmax)
    n2 = ofit.applied_norm2(psi0, Wo)
    eps_or = 1.0 - r1["norm"] ** 2 / n2
    z_or = ofit.expect_local(ref1, wl.SZ, LR_SITE).real
    out = {"step1": {"oracle_norm": r1["norm"], "oracle_eps": eps_or, "W_psi0_norm2": n2,
                     "oracle_max_bond": max(r1["bond_dims"])}}
    dpsi0 = mp.DeviceMPS(psi0, Dmax=Dmax)
    for name, p in (("fp32", mp.FP32), ("fp64", mp.FP64), ("bf16x3", mp.BF16X3)):
        dm = mp.DeviceMPS(psi0, Dmax=Dmax)
        s = mp.step(h, dm, dw, prec=p)
        phi = dm.to_numpy()
        # eps of the device state from its FP64 overlap with W psi0 (the norms and overlaps in FP64)
        eps = 1.0 - abs(mp.overlap(h, dm, dw, dpsi0)) ** 2 / n2
        out["step1"][name] = {"infidelity_R17A": float(1.0 - abs(ofit.overlap(phi, ref1)) ** 2),
                              "eps_excess_R17B": float(abs(eps - eps_or)),
                              "eps_excess_from_step_norm": float(abs(1.0 - s.norm ** 2 / n2 - eps_or)),
                              "Z50_error": float(abs(ofit.expect_local(phi, wl.SZ, LR_SITE).real - z_or)),
                              "norm_rel_error": float(abs(s.norm - r1["norm"]) / r1["norm"])}
        del dm
    # step 1 from the zip-up of W psi0 (bonds up to Dmax before the sweeps; its oracle parity is a
    # GPU test at L = 8, the oracle's zip-up fit at this size takes a minute)
    zs = {}
    for name, p in (("fp32", mp.FP32), ("fp64", mp.FP64)):
        dm = mp.DeviceMPS(psi0, Dmax=Dmax)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s = mp.step(h, dm, dw, prec=p, guess=mp.GUESS_ZIPUP)
        torch.cuda.synchronize()
        zs[name] = {"ms": (time.perf_counter() - t1) * 1e3, "max_bond": s.max_bond,
                    "eps": float(1.0 - abs(mp.overlap(h, dm, dw, dpsi0)) ** 2 / n2),
                    "norm": s.norm}
        del dm
    zs["oracle_eps_canonical_guess"] = eps_or
    out["step1_zipup_guess"] = zs
    if delta2:
        if nsites == -1:
            ref2, r2 = ofit.fit_step_mixed(ref1, Wo, Dmax=Dmax)
        elif nsites == 1:
            ref2, r2 = ofit.fit_step_one_site(ref1, Wo)
            r2["discarded"] = [0.0]
        else:
            ref2, r2 = ofit.fit_step(ref1, Wo, Dmax=Dmax)
        z2 = ofit.expect_local(ref2, wl.SZ, LR_SITE).real
        out["step2_from_oracle_state"] = {"oracle_norm": r2["norm"], "oracle_max_bond": max(r2["bond_dims"]),
                                          "oracle_discarded_sum": float(sum(r2["discarded"])),
                                          "nsites": nsites,
                                          "oracle_one_site_visits": r2.get("kinds", []).count(1)}
        for name, p in (("fp32", mp.FP32), ("fp64", mp.FP64)):
            dm = mp.DeviceMPS(ref1, Dmax=Dmax)
            s = mp.step(h, dm, dw, prec=p, nsites=nsites)
            phi = dm.to_numpy()
            out["step2_from_oracle_state"][name] = {
                "one_site_visits": s.one_site_visits,
                "infidelity_R17A": float(1.0 - abs(ofit.overlap(phi, ref2)) ** 2),
                "norm_rel_error": float(abs(s.norm - r2["norm"]) / r2["norm"]),
                "discarded_sum_abs_error": float(abs(s.discarded_sum - sum(r2["discarded"]))),
                "Z50_error": float(abs(ofit.expect_local(phi, wl.SZ, LR_SITE).real - z2))}
            del dm
    out["oracle_wall_s"] = time.perf_counter() - t0
    torch.cuda.empty_cache()
    return out


def lr3_cpu_baseline(Wo, wl, Dmax, visits=4):
    """The oracle timed on a bounded sample of the workload: `visits` bond visits at saturated
    bond dimension (seeded random environments and sites, D = 256, w = 271): the projected
    two-site tensor, its FP64 SVD truncation and one environment update, scaled to the
    4 (L - 1) visits of a step (extrapolated)."""
    from oracle import fit as ofit
    import threadpoolctl
    rng = np.random.default_rng(1)
    w = Wo.shape[0]
    t = 0.0
    for _ in range(visits):
        Lenv = wl.complex_normal(rng, (Dmax, w, Dmax))
        Renv = wl.complex_normal(rng, (Dmax, w, Dmax))
        M1, M2 = wl.complex_normal(rng, (Dmax, 2, Dmax)), wl.complex_normal(rng, (Dmax, 2, Dmax))
        t0 = time.perf_counter()
        th = ofit.theta_two_site(Lenv, M1, Wo, M2, Wo, Renv)
        U, S, Vh, _ = ofit.svd_truncate(th.reshape(2 * Dmax, 2 * Dmax), Dmax, 1e-14)
        ofit.env_left(Lenv, U.reshape(Dmax, 2, -1), Wo, M1)
        t += time.perf_counter() - t0
    per_visit = t / visits
    info = threadpoolctl.threadpool_info()
    threads = max([i.get("num_threads", 1) for i in info] + [1])
    nv = 4 * (LR_L - 1)
    return {"value": per_visit * nv, "unit": "s per time step (extrapolated, saturated bonds)",
            "cores": int(threads), "kind": "oracle",
            "sample": f"{visits} bond visits of the oracle at saturated bond dimension (D={Dmax}, w={w}, seeded "
                      f"random environments and sites): projected two-site tensor, FP64 SVD truncation of the "
                      f"{2 * Dmax}x{2 * Dmax} matrix, one environment update; {per_visit:.2f} s per visit "
                      f"(numpy complex128, {threads} BLAS threads), times the {nv} visits of a step",
            "sample_wall_s": t}


def run_lr3(args, torch, mp, wl, h):
    """The default line: K steps of the long-range Ising chain from all-up (see the module
    docstring), FP32 products against plain FP64 on the same opening steps."""
    from oracle import mpo as ompo
    K, Wm = args.steps, args.warmup
    prec = prec_of(mp, args.prec)
    H = lr_blocks(wl)
    W, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, LR_ORDER, -1j * LR_TAU, mp.V2_EXTENDED)
    w = W.shape[0]
    dw = mp.DeviceMPO([W] * LR_L)
    psi0 = wl.all_up(LR_L)
    prog = "lr3" if args.progress else None
    ns = args.nsites
    # a step whose plan the handle has seen before (the warm-up steps are the first sightings) is
    # captured into a HIP graph and replayed, unless --no-graph
    gs, gr = guess_of(mp, args), not args.no_graph
    # the environment microbenchmark first, on a device that has not yet run minutes of work
    envmb = None if args.no_side else env_microbench_summary(mp, h, torch)
    # the tile tuner times the products of the shapes the warm-up steps meet and keeps the fastest
    # plan; frozen for the timed steps (shapes it has not seen take the planner's rule)
    tune = args.tune
    if tune:
        h.set_tuning(mp.TUNE_ON)
    if Wm:  # untimed warm-up steps of the same trajectory on their own state and workspace
        trajectory(torch, mp, h, psi0, dw, prec, Wm, LR_D, progress=prog and prog + " warm-up", nsites=ns,
                   guess=gs, use_graph=gr)
    if tune:
        h.set_tuning(mp.TUNE_FROZEN)
    ms, st, dm = trajectory(torch, mp, h, psi0, dw, prec, K, LR_D, profile=not gr, progress=prog, nsites=ns,
                            guess=gs, use_graph=gr)
    graph_steps = [i + 1 for i, x in enumerate(st) if x.graph]
    if gr:  # the kernel table from the same steps profiled launch by launch (untimed)
        _, st, dmp = trajectory(torch, mp, h, psi0, dw, prec, K, LR_D, profile=True, nsites=ns, guess=gs)
        del dmp
    sec = float(np.sum(ms)) / 1e3 / K
    kt = kernel_table(st, args.prec)
    prof = {k: float(sum(x.profile[k] for x in st)) for k in st[0].profile if k != "kernels"}
    gemm_tf = prof["gemm_gflop"] / prof["t_gemm_ms"] if prof["t_gemm_ms"] > 0 else 0.0
    Id = np.eye(2, dtype=np.complex128).reshape(1, 2, 2, 1)
    zops = [Id] * LR_L
    zops[LR_SITE] = wl.SZ.reshape(1, 2, 2, 1)
    dZ = mp.DeviceMPO(zops)
    z_end = mp.expectation(h, dm, dZ).real
    sat = [i for i, x in enumerate(st) if x.max_bond >= LR_D]
    fp64 = None
    if not args.no_fp64 and prec != mp.FP64:
        n64 = max(1, min(args.fp64_steps or K, K))
        if tune:  # the same warm-up and tuning for the FP64 path's products
            h.set_tuning(mp.TUNE_ON)
            if Wm:
                trajectory(torch, mp, h, psi0, dw, mp.FP64, Wm, LR_D, progress=prog and prog + " fp64 warm-up",
                           nsites=ns, guess=gs)
            h.set_tuning(mp.TUNE_FROZEN)
        ms64, st64, dm64 = trajectory(torch, mp, h, psi0, dw, mp.FP64, n64, LR_D, profile=True,
                                      progress=prog and prog + " fp64", nsites=ns, guess=gs)
        p64 = {k: float(sum(x.profile[k] for x in st64)) for k in st64[0].profile if k != "kernels"}
        fp64 = {"steps": n64, "launches": "kernel by kernel, each timed (no graphs)",
                "fp64_s_per_step": float(np.sum(ms64)) / 1e3 / n64,
                "fp32_s_per_step_same_steps": float(np.sum(ms[:n64])) / 1e3 / n64,
                "fp64_gemm_tflops": p64["gemm_gflop"] / p64["t_gemm_ms"] if p64["t_gemm_ms"] > 0 else 0.0,
                "fp64_jacobi_share": p64["t_jacobi_ms"] / max(float(np.sum(ms64)), 1e-9),
                "fp64_dominant_kernel": roofline_of(kernel_table(st64, "fp64")[0])}
        fp64["fp32_speedup"] = fp64["fp64_s_per_step"] / fp64["fp32_s_per_step_same_steps"]
        if n64 == K:  # the two trajectories after the same K steps from psi0
            a, b = dm.to_numpy(), dm64.to_numpy()
            fp64["trajectory_infidelity_fp32_vs_fp64"] = float(1.0 - abs(_overlap(a, b)) ** 2 / (
                abs(_overlap(a, a)) * abs(_overlap(b, b))))
            fp64["Z50_end_fp32"] = z_end
            fp64["Z50_end_fp64"] = mp.expectation(h, dm64, dZ).real
            fp64["Z50_abs_diff"] = abs(fp64["Z50_end_fp32"] - fp64["Z50_end_fp64"])
        del dm64
        torch.cuda.empty_cache()
    del dm
    torch.cuda.empty_cache()
    parity = cpu = None
    if not args.no_cpu:
        Wo = ompo.build_mpo(H, LR_ORDER, -1j * LR_TAU, "V2")
        if prog:
            print("[bench] lr3 parity against the oracle (steps 1 and 2)", file=sys.stderr, flush=True)
        parity = lr3_parity(torch, mp, h, wl, W, Wo, dw, psi0, LR_D, delta2=not args.no_delta2, nsites=ns)
        if prog:
            print("[bench] lr3 CPU oracle baseline", file=sys.stderr, flush=True)
        cpu = lr3_cpu_baseline(Wo, wl, LR_D)
    if prog and not args.no_side:
        print("[bench] side field: quench steps 1-20", file=sys.stderr, flush=True)
    side = {} if args.no_side else {"quench_L64_D128": run_quench(args, torch, mp, wl, h, side=True),
                                    "env_microbench": envmb}
    line = {
        "metric": "s per time step & TFLOP/s at D=256: FP32-MFMA grouped vs plain FP64, fidelity",
        "value": sec, "unit": "s per time step", "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": sec * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[args.prec], "data": "synthetic",
        "config": {"workload": f"long-range Ising L={LR_L}, J(r)=r^-2 as 6 exponentials, g=1, order-{LR_ORDER} "
                               f"extended MPO (w={w}), tau={LR_TAU} (real time), D<={LR_D}, all-up start, "
                               f"2 sweeps per step ({NSITES_DESC[ns]}){GUESS_DESC[args.guess]}"
                               f"{', steps replayed from HIP graphs' if gr else ''}, steps 1..{K} from t=0",
                   "L": LR_L, "D": LR_D, "order": LR_ORDER, "tau": LR_TAU, "w": w},
        "step_ms": ms,
        "graph_steps": graph_steps if gr else None,
        "tile_tuner": ({"mode": "timed the product plans of the warm-up steps' shapes (FP32 and FP64 each), "
                                "frozen for the timed steps", "entries": h.product_plan(prec, 1, 1, 1)["entries"]}
                       if tune else None),
        "max_bond_per_step": [x.max_bond for x in st],
        "one_site_steps": [i + 1 for i, x in enumerate(st) if x.one_site_visits == x.visits],
        "mixed_steps": {i + 1: f"{x.one_site_visits}/{x.visits} one-site visits" for i, x in enumerate(st)
                        if 0 < x.one_site_visits < x.visits},
        "discarded_sum_per_step": [x.discarded_sum for x in st],
        "saturated_steps": len(sat),
        "saturated_s_per_step": float(np.mean([ms[i] for i in sat])) / 1e3 if sat else None,
        "step_tflop_mean": float(np.mean([x.gflop for x in st])) / 1e3,
        "products_tflops": gemm_tf,
        "products_frac_of_peak": gemm_tf * 1e12 / {mp.FP32: PEAK_FP32_MFMA, mp.FP64: PEAK_FP64_MFMA,
                                                   mp.BF16X3: PEAK_BF16_MFMA}[prec],
        "class_ms_timed_steps": {"jacobi_svd": prof["t_jacobi_ms"], "complex_gemm": prof["t_gemm_ms"],
                                 "w_contraction": prof["t_wmix_ms"],
                                 "householder_qr": float(sum(r["ms"] for r in kt if r["kind"] == "householder_qr")),
                                 "all_steps": float(np.sum(ms))},
        # Jacobi sweeps per two-site truncation (one-site visits take none)
        "svd_sweeps_mean": float(sum(x.svd_sweeps_total for x in st) /
                                 max(sum(x.visits - x.one_site_visits for x in st), 1)),
        "Z50_end": z_end,
        "roofline": roofline_of(kt[0]),
        "kernels_timed_steps": kt[:8],
        "fp64_path": fp64,
        "parity_vs_oracle": parity,
        **side,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def env_microbench_summary(mp, h, torch):
    mb32_ms, mb_flop = env_microbench(mp, h, torch, mp.FP32)
    mb64_ms, _ = env_microbench(mp, h, torch, mp.FP64)
    mbbf_ms, _ = env_microbench(mp, h, torch, mp.BF16X3)
    tf32 = mb_flop / (mb32_ms * 1e-3) / 1e12
    return {"D": 256, "d": 2, "w": 8, "flop_per_call": mb_flop,
            "fp32_ms": mb32_ms, "fp32_tflops": tf32,
            "fp32_frac_of_mfma_peak": tf32 * 1e12 / PEAK_FP32_MFMA,
            "fp32_executed_frac_of_mfma_peak": 0.75 * tf32 * 1e12 / PEAK_FP32_MFMA,
            "fp64_ms": mb64_ms, "fp64_tflops": mb_flop / (mb64_ms * 1e-3) / 1e12,
            "fp64_frac_of_mfma_peak": mb_flop / (mb64_ms * 1e-3) / PEAK_FP64_MFMA,
            "bf16x3_ms": mbbf_ms, "bf16x3_tflops": mb_flop / (mbbf_ms * 1e-3) / 1e12,
            "bf16x3_frac_of_ceiling": mb_flop / (mbbf_ms * 1e-3) / CEIL_BF16X3}


def run_env(args, torch, mp, h):
    """The environment-update microbenchmark alone: FP32 (three real products per complex
    multiply-add on the fp32 matrix cores), plain FP64 and split-BF16x3, K calls each."""
    reps = max(1, args.steps or (100 if args.env_w == 8 else 10))
    w = args.env_w
    res = {}
    for name in ("fp32", "fp64", "bf16x3"):
        ms, flop = env_microbench(mp, h, torch, prec_of(mp, name), reps=reps, w=w)
        peak = 78.6 if name == "fp64" else 157.3
        res[name] = {"us": ms * 1e3, "tflops": flop / ms / 1e9, "frac_of_peak": flop / ms / 1e9 / peak,
                     "peak_tflops": peak}
    f32 = res["fp32"]
    opd = ("W (8, 2, 2, 8), seeded complex normal operands" if w == 8 else
           f"W the long-range chain's order-3 MPO ({w}, 2, 2, {w}), seeded complex normal E and sites")
    print(json.dumps({
        "metric": f"env_update (left) TFLOP/s at D=256, d=2, w={w}, FP32 matrix cores",
        "value": f32["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": reps, "warmup": env_warmup(w),
        "ms_per_step": f32["us"] / 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"left environment update, E (256, {w}, 256), ket/bra (256, 2, 256), " + opd,
                   "flop_per_call": 8.0 * (2 * 256 ** 3 * 2 * w + 256 ** 2 * 2 ** 2 * w ** 2)},
        "roofline": {"bound": "mfma", "achieved": f32["tflops"], "peak": 157.3, "unit": "TFLOP/s",
                     "frac": f32["frac_of_peak"], "traffic": None},
        "precisions": res,
    }), flush=True)


def run_copy(args, torch):
    """Calibration of the HBM counters: a plain device copy of 256 MiB, K times (torch's copy
    kernel); FETCH_SIZE and WRITE_SIZE per dispatch against the 256 MiB it reads and writes give
    the scale factors of the counter tables in profiles/."""
    n = 256 * 2 ** 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    reps = max(1, args.steps or 10)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        dst.copy_(src)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    print(json.dumps({"metric": "device copy bandwidth (counter calibration)", "value": 2 * n / ms / 1e6,
                      "unit": "GB/s", "n_gpus": 1, "steps": reps, "warmup": 0, "ms_per_step": ms,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
                      "data": "synthetic", "config": {"workload": "device copy of 256 MiB", "bytes": n},
                      "roofline": {"bound": "hbm", "achieved": 2 * n / ms / 1e6, "peak": PEAK_HBM / 1e9,
                                   "unit": "GB/s", "frac": 2 * n / ms / 1e6 / (PEAK_HBM / 1e9),
                                   "traffic": 2 * n}}), flush=True)


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
    steps = args.steps or 20
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
    steps = args.steps or 20
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
    steps = args.steps or 3
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
        ms, first, graphs = [], None, []
        for k in range(steps):
            t0 = time.perf_counter()
            if batched:
                st = mp.step_batched(h, dms, dws, prec=prec, workspace=ws, input_right_canonical=k > 0,
                                     use_graph=args.graph)
            else:
                st = [mp.step(h, dm, dw, prec=prec, workspace=w_, input_right_canonical=k > 0)
                      for dm, dw, w_ in zip(dms, dws, ws)]
            graphs.append(sum(1 for x in st if x.graph == 2))
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
            if k == 0:
                first = [dm.to_numpy() for dm in dms[:4]]
        bonds = [max(dm.bond) for dm in dms]
        gflop = sum(x.gflop for x in st)
        del ws, dms
        torch.cuda.empty_cache()
        return ms, first, bonds, gflop, graphs

    ms_b, first_b, bonds, gflop, graphs_b = trajectory(True)
    ms_1, first_1, _, _, _ = trajectory(False)
    sec = float(np.sum(ms_b)) / 1e3 / steps
    parity, cpu = None, None
    if not args.no_cpu:
        from oracle import fit as ofit
        from oracle import mpo as ompo
        import threadpoolctl
        parity = []
        t0 = time.perf_counter()
        for c in range(4):
            g, Lc, Dc = chains[c]
            ref, _ = ofit.fit_step(wl.all_up(Lc), ompo.build_mpo(wl.tfim(g), 2, -1j * TAU, "V2"), Dmax=Dc,
                                   nsweeps=2)
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
                               f"2 sweeps, all-up start, steps 1..{steps}"
                               f"{', each chain replaying its captured step graph once its plan repeats' if args.graph else ''}",
                   "chains": len(chains), "tau": TAU, "order": 2},
        "steps_ms_batched": ms_b, "steps_ms_one_by_one": ms_1,
        "graph_replays_per_step": graphs_b if args.graph else None,
        "batched_speedup": float(np.sum(ms_1) / np.sum(ms_b)),
        "chain_steps_per_s": len(chains) * steps / (float(np.sum(ms_b)) / 1e3),
        "worker_streams_requested": int(os.environ.get("MPOEVO_BATCH_STREAMS", "4")),
        "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"),
        "last_step_gflop": gflop, "max_bond_per_chain_end": bonds,
        "parity_vs_oracle": parity,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


XXZ_L, XXZ_UP, XXZ_D, XXZ_ORDER, XXZ_TAU, XXZ_DELTA = 128, 64, 512, 2, 0.1, 0.5


def run_xxz(args, torch, mp, wl, h, side=False):
    """The XXZ chain with U(1) charges (configuration 4): L = 128, 64 up spins, Delta = 0.5, the
    order-2 extended MPO (w = 13), tau = 0.1, D <= 512 over about 15 charge sectors per bond (the
    seeded sector tables of the input recipe, seed 1), K steps (default 20; side=True: 3) from
    the seeded random U(1) state, FP32 and FP64; the oracle's block-sparse step 1 for parity."""
    K = 3 if side else (args.steps or 20)
    H = wl.xxz(XXZ_DELTA)
    qp = H.phys_charge
    W, lc = mp.mpo_build(H.A, H.B, H.C, H.Dloc, XXZ_ORDER, -1j * XXZ_TAU, mp.V2_EXTENDED, H.inner_charge, qp)
    tables = wl.u1_sector_tables(XXZ_L, XXZ_UP, XXZ_D, nsec=15, seed=1)
    psi = wl.random_u1_mps(np.random.default_rng(1), tables, qp)
    dense, charges = wl.u1_dense(psi, tables, qp)
    dw = mp.DeviceMPO([W] * XXZ_L)
    prog = "xxz" if args.progress else None

    def run(prec, n, profile=False):
        dm = mp.DeviceMPS(dense, Dmax=XXZ_D, charges=charges, phys_charge=qp)
        ws = mp.step_workspace(dm, dw, prec)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
        st = []
        torch.cuda.synchronize()
        ev[0].record()
        for k in range(n):
            st.append(mp.step(h, dm, dw, prec=prec, input_right_canonical=k > 0, workspace=ws, profile=profile))
            ev[k + 1].record()
            if prog:
                print(f"[bench] {prog} prec {prec} step {k + 1}/{n}: bond {st[-1].max_bond}", file=sys.stderr,
                      flush=True)
        torch.cuda.synchronize()
        del ws
        torch.cuda.empty_cache()
        return [ev[k].elapsed_time(ev[k + 1]) for k in range(n)], st, dm

    prec = mp.FP32 if side else prec_of(mp, args.prec)
    if not side and args.warmup:
        run(prec, min(args.warmup, 2))
    ms, st, dm = run(prec, K, profile=True)
    sec = float(np.sum(ms)) / 1e3 / K
    kt = kernel_table(st, "fp32" if side else args.prec)
    nsec = [len(set(c)) for c in dm.charges[1:-1]]
    out = {"workload": f"XXZ chain (Delta={XXZ_DELTA}) with U(1) charges, L={XXZ_L}, {XXZ_UP} up spins, order-"
                       f"{XXZ_ORDER} extended MPO (w={W.shape[0]}), tau={XXZ_TAU}, D<={XXZ_D} over charge sectors "
                       f"(seeded tables, seed 1), steps 1..{K} from the seeded random U(1) state",
           "s_per_step": sec, "step_ms": ms, "max_bond_end": max(dm.bond), "sectors_per_bond_end_max": max(nsec),
           "discarded_sum_per_step": [x.discarded_sum for x in st],
           "products_ms": float(sum(x.profile["t_gemm_ms"] for x in st)),
           "dominant_kernel": roofline_of(kt[0]) if kt else None}
    if not (side or args.no_fp64) and prec != mp.FP64:
        ms64, _, dm64 = run(mp.FP64, K)
        a, b = dm.to_numpy(), dm64.to_numpy()
        out["fp64_s_per_step"] = float(np.sum(ms64)) / 1e3 / K
        out["fp32_speedup"] = out["fp64_s_per_step"] / sec
        out["trajectory_infidelity_fp32_vs_fp64"] = float(1.0 - abs(_overlap(a, b)) ** 2 / (
            abs(_overlap(a, a)) * abs(_overlap(b, b))))
        del dm64
    del dm
    torch.cuda.empty_cache()
    if not side and not args.no_cpu:
        from oracle import mpo as ompo
        from oracle import u1 as ou1
        Wo = ompo.build_mpo(H, XXZ_ORDER, -1j * XXZ_TAU, "V2")
        lco = ompo.level_charges(H, XXZ_ORDER, -1j * XXZ_TAU, "V2")
        t0 = time.perf_counter()
        ref, rb, rst = ou1.fit_step(psi, tables, Wo, lco, qp, Dmax=XXZ_D)
        t_or = time.perf_counter() - t0
        refd = ou1.to_dense(ref, rb, qp)
        par = {}
        for name, p in (("fp32", mp.FP32), ("fp64", mp.FP64)):
            dm1 = mp.DeviceMPS(dense, Dmax=XXZ_D, charges=charges, phys_charge=qp)
            s1 = mp.step(h, dm1, dw, prec=p)
            par[name] = {"step1_infidelity_R17A": float(1.0 - abs(_overlap(dm1.to_numpy(), refd)) ** 2),
                         "step1_norm_rel_error": float(abs(s1.norm - rst["norm"]) / rst["norm"]),
                         "step1_discarded_abs_error": float(abs(s1.discarded_sum - sum(rst["discarded"]))),
                         "bond_charges_equal": all(sorted(dm1.charges[b]) ==
                                                   [q for q in sorted(rb[b]) for _ in range(rb[b][q])]
                                                   for b in range(XXZ_L + 1))}
            del dm1
        out["parity_vs_block_oracle"] = par
        import threadpoolctl
        threads = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] + [1])
        out["cpu_baseline"] = {"value": t_or, "unit": "s per time step", "cores": int(threads), "kind": "oracle",
                               "sample": "the block-sparse oracle's step 1 from the same state (dictionaries of "
                                         f"blocks, numpy complex128, {threads} BLAS threads)"}
    if side:
        return out
    print(json.dumps({
        "metric": "s per time step, U(1) XXZ chain (configuration 4)",
        "value": sec, "unit": "s per time step", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[args.prec], "data": "synthetic",
        "config": {"workload": out["workload"], "L": XXZ_L, "D": XXZ_D, "order": XXZ_ORDER, "tau": XXZ_TAU},
        "roofline": out["dominant_kernel"], "kernels_timed_steps": kt[:8],
        **{k: v for k, v in out.items() if k not in ("workload", "dominant_kernel")}}), flush=True)


def run_quench(args, torch, mp, wl, h, side=False):
    """The L = 64 TFIM quench (g = 0.5 -> 1.5) from t = 0: K steps on the chosen path and the same
    steps on the plain FP64 path, first-step parity against the oracle (R17-A and R17-B), the
    dominant kernel. side=True: steps 1..20 on the FP32 path, returned as a dict."""
    from oracle import fit as ofit
    from oracle import mpo as ompo
    steps = 20 if side else (args.steps or 100)
    prec = mp.FP32 if side else prec_of(mp, args.prec)
    pname = "fp32" if side else args.prec
    psi0 = load_ground()
    H = wl.tfim(G_AFTER)
    W, _ = mp.mpo_build(H.A, H.B, H.C, H.Dloc, ORDER, -1j * TAU, mp.V2_EXTENDED)
    dw = mp.DeviceMPO([W] * L)
    prog = ("quench" if args.progress else None)
    gs, gr = (0, False) if side else (guess_of(mp, args), args.graph)
    if not side and args.warmup:
        trajectory(torch, mp, h, psi0, dw, prec, args.warmup, D, guess=gs, use_graph=gr)
    ms, st, dm = trajectory(torch, mp, h, psi0, dw, prec, steps, D, profile=not gr, progress=prog, guess=gs,
                            use_graph=gr)
    if gr:  # the kernel table from the same steps profiled launch by launch (untimed)
        _, st, dmp = trajectory(torch, mp, h, psi0, dw, prec, steps, D, profile=True, guess=gs)
        del dmp
    sec = float(np.sum(ms)) / 1e3 / steps
    kt = kernel_table(st, pname)
    Id = np.eye(2, dtype=np.complex128).reshape(1, 2, 2, 1)
    zops = [Id] * L
    zops[31] = wl.SZ.reshape(1, 2, 2, 1)
    dZ = mp.DeviceMPO(zops)
    out = {"workload": f"TFIM quench L={L} from the g=0.5 ground state to g={G_AFTER}, order-{ORDER} extended "
                       f"MPO (w={W.shape[0]}), tau={TAU}, D<={D}"
                       f"{'' if side else GUESS_DESC[args.guess]}"
                       f"{', steps replayed from HIP graphs' if gr else ''}, steps 1..{steps} from t=0",
           "s_per_step": sec, "steps": steps, "max_bond_last_step": st[-1].max_bond,
           "dominant_kernel": roofline_of(kt[0])}
    if (side or not args.no_fp64) and prec != mp.FP64:
        ms64, _, dm64 = trajectory(torch, mp, h, psi0, dw, mp.FP64, steps, D, guess=gs, use_graph=gr)
        a, b = dm.to_numpy(), dm64.to_numpy()
        out["fp64_s_per_step"] = float(np.sum(ms64)) / 1e3 / steps
        out["fp32_speedup"] = out["fp64_s_per_step"] / sec
        out["trajectory_infidelity_fp32_vs_fp64"] = float(1.0 - abs(_overlap(a, b)) ** 2 / (
            abs(_overlap(a, a)) * abs(_overlap(b, b))))
        out["Z32_abs_diff_fp32_vs_fp64"] = abs(mp.expectation(h, dm, dZ).real - mp.expectation(h, dm64, dZ).real)
        del dm64
    del dm
    torch.cuda.empty_cache()
    if not args.no_cpu:
        Wo = ompo.build_mpo(H, ORDER, -1j * TAU, "V2")
        ref, rinfo = ofit.fit_step(psi0, Wo, Dmax=D)
        n2 = ofit.applied_norm2(psi0, Wo)
        eps_or = 1.0 - rinfo["norm"] ** 2 / n2
        z_or = ofit.expect_local(ref, wl.SZ, 31).real
        par = {}
        dpsi0 = mp.DeviceMPS(psi0, Dmax=D)
        for name, p in (("fp32", mp.FP32), ("fp64", mp.FP64), ("bf16x3", mp.BF16X3)):
            dm1 = mp.DeviceMPS(psi0, Dmax=D)
            s1 = mp.step(h, dm1, dw, prec=p)
            o = dm1.to_numpy()
            eps = 1.0 - abs(mp.overlap(h, dm1, dw, dpsi0)) ** 2 / n2
            par[name] = {"infidelity_R17A": float(1.0 - abs(ofit.overlap(o, ref)) ** 2),
                         "eps_excess_R17B": float(abs(eps - eps_or)),
                         "eps_excess_from_step_norm": float(abs(1.0 - s1.norm ** 2 / n2 - eps_or)),
                         "Z32_error": float(abs(ofit.expect_local(o, wl.SZ, 31).real - z_or)),
                         "norm_rel_error": float(abs(s1.norm - rinfo["norm"]) / rinfo["norm"])}
        out["step1_parity_vs_oracle"] = par
    if side:
        return out
    print(json.dumps({
        "metric": "s per time step, TFIM quench L=64 (configuration 2)",
        "value": sec, "unit": "s per time step", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[args.prec], "data": "synthetic",
        "config": {"workload": out["workload"], "L": L, "D": D, "order": ORDER, "tau": TAU},
        "step_ms": ms, "roofline": out["dominant_kernel"], "kernels_timed_steps": kt[:8],
        **{k: v for k, v in out.items() if k not in ("workload", "dominant_kernel")}}), flush=True)


def main():
    global ORDER, TAU
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 20 for lr3, 100 for quench, 3 for batched, 20 for split/thermal, "
                         "100 calls for env)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed warm-up steps (default 2; 1 for quench)")
    ap.add_argument("--prec", choices=["fp32", "fp64", "bf16x3"], default="fp32")
    ap.add_argument("--fp64-steps", type=int, default=None, help="opening steps run on the FP64 path too (default: all)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and parity")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--no-delta2", action="store_true", help="lr3: skip the step-2 parity from the oracle state")
    ap.add_argument("--no-side", action="store_true", help="lr3: skip the quench and microbenchmark side fields")
    ap.add_argument("--tune", action="store_true",
                    help="lr3: tune the product plans on the warm-up steps, frozen for the timed steps (default: the "
                         "planner's rule)")
    ap.add_argument("--nsites", type=int, default=-1, choices=[-1, 1, 2],
                    help="lr3: local update (2: two-site; 1: one-site at fixed bonds; -1: two-site while the "
                         "bonds grow, one-site once all are at their largest value)")
    ap.add_argument("--workload", choices=["lr3", "quench", "xxz", "batched", "env", "split", "thermal",
                                           "cylinder", "copy"], default="lr3")
    ap.add_argument("--progress", action="store_true", default=True,
                    help="print a line to stderr after every timed step and phase (the default)")
    ap.add_argument("--quiet", dest="progress", action="store_false", help="no progress lines on stderr")
    ap.add_argument("--env-w", type=int, default=8, choices=[8, 271],
                    help="env workload: the MPO bond (8: the microbenchmark; 271: the long-range chain's MPO)")
    ap.add_argument("--guess", choices=["canonical", "zipup", "auto"], default="canonical",
                    help="lr3 and quench: the sweeps' starting point (psi, the zip-up of W psi, or the zip-up "
                         "while the bonds grow)")
    ap.add_argument("--graph", action="store_true",
                    help="quench and batched: replay each step's launches from a captured HIP graph once its "
                         "plan repeats (lr3 does by default)")
    ap.add_argument("--no-graph", action="store_true",
                    help="lr3: launch every step's kernels one by one instead of replaying a step whose plan was "
                         "seen before from its captured HIP graph")
    ap.add_argument("--order", type=int, default=ORDER, choices=[1, 2, 3, 4],
                    help="MPO order of the TFIM workloads (quench, split reference, thermal)")
    ap.add_argument("--tau", type=float, default=TAU, help="time step of the quench and split workloads")
    args = ap.parse_args()
    ORDER, TAU = args.order, args.tau
    if args.warmup is None:
        args.warmup = 1 if args.workload == "quench" else 2
    if args.workload == "lr3" and args.steps is None:
        args.steps = 20
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
    if args.workload == "copy":
        run_copy(args, torch)
        return
    h = mp.Handle(0)
    if args.workload == "env":
        run_env(args, torch, mp, h)
    elif args.workload == "quench":
        run_quench(args, torch, mp, wl, h)
    else:
        {"lr3": run_lr3, "xxz": run_xxz, "batched": run_batched, "split": run_split, "thermal": run_thermal,
         "cylinder": run_cylinder}[args.workload](args, torch, mp, wl, h)
    h.close()


if __name__ == "__main__":
    main()
