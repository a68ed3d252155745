"""Writes tfim_g05_L64_ground.npz, the initial state of the L = 64 transverse-field Ising quench:
the ground state of H = -sum Z_i Z_{i+1} - g sum X_i at g = 0.5 on an open chain of 64 sites.

It is prepared by the oracle alone: imaginary-time evolution with the order-2 extended MPO of
exp(tau H) at real tau = -0.05 (Sec. 3 and Sec. 5 of the paper; the same MPO family as the real-time
steps, with tau real), two-site variational fits with bond dimension at most 128 and the
truncation rule of the fit, starting from the all-up product state, until the energy per step
changes by less than 1e-12. Run from the repository root:  python tests/golden/make_tfim_ground.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fit, mpo  # noqa: E402
from paper_2302_14181_amd import workloads as wl  # noqa: E402

L, G, TAU, ORDER, DMAX, TOL, MAX_STEPS = 64, 0.5, -0.05, 2, 128, 1e-12, 4000
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tfim_g05_L64_ground.npz")


def energy(ms, H) -> float:
    Wh = mpo.hamiltonian_mpo(H)
    w = Wh.shape[0]
    left = np.zeros(w, dtype=np.complex128)
    right = np.zeros(w, dtype=np.complex128)
    left[0] = 1.0
    right[w - 1] = 1.0
    return float((fit.mpo_expectation(ms, [Wh] * len(ms), left, right) / fit.overlap(ms, ms)).real)


def main():
    H = wl.tfim(G)
    W = mpo.build_mpo(H, ORDER, TAU, "V2")
    psi = wl.all_up(L)
    e_prev = energy(psi, H)
    t0 = time.time()
    for step in range(1, MAX_STEPS + 1):
        psi, _ = fit.fit_step(psi, W, DMAX, nsweeps=2)
        e = energy(psi, H)
        if step % 20 == 0:
            print(f"step {step} E={e:.15f} dE={e - e_prev:.2e} maxD={max(m.shape[2] for m in psi)} "
                  f"{time.time() - t0:.0f}s", flush=True)
        if abs(e - e_prev) < TOL:
            break
        e_prev = e
    else:
        raise SystemExit("imaginary-time evolution did not settle")
    np.savez_compressed(OUT, **{f"site_{i:03d}": m for i, m in enumerate(psi)},
                        energy=np.float64(e), steps=np.int64(step), g=np.float64(G), tau=np.float64(TAU))
    print(f"wrote {OUT}: steps={step} E={e:.15f} bonds={[m.shape[2] for m in psi[:-1]]}")


if __name__ == "__main__":
    main()
