"""Writes lr_fit_K6.json: the couplings of the long-range Ising input, J(r) = r^-2 on r = 1..99
approximated by a sum of K = 6 exponentials, J(r) ~ sum_k c_k lambda_k^(r-1) (the form the
Jordan-block Hamiltonians of Sec. 2.3 need for long-range interactions).

Matrix-pencil method (Hua and Sarkar): the Hankel matrix of the samples, its K dominant right
singular vectors V, the poles lambda_k as the eigenvalues of pinv(V[:-1]) V[1:], then the
amplitudes c_k by linear least squares on all samples. numpy only. Run from the repository root:
python tests/golden/make_lr_fit.py
"""
import json
import os

import numpy as np

ALPHA, K, RMAX = 2.0, 6, 99
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lr_fit_K6.json")


def fit(alpha=ALPHA, k=K, rmax=RMAX):
    r = np.arange(1, rmax + 1, dtype=np.float64)
    y = r ** (-alpha)
    pencil = rmax // 3
    Y = np.array([y[i:i + pencil + 1] for i in range(rmax - pencil)])
    _, _, vh = np.linalg.svd(Y, full_matrices=False)
    V = vh[:k].T
    lam = np.linalg.eigvals(np.linalg.pinv(V[:-1]) @ V[1:])
    lam = np.sort(lam.real)[::-1]
    vander = lam[None, :] ** (r[:, None] - 1)
    c, *_ = np.linalg.lstsq(vander, y, rcond=None)
    err = np.max(np.abs(vander @ c - y) / y)
    return c, lam, float(err)


if __name__ == "__main__":
    c, lam, err = fit()
    json.dump({"alpha": ALPHA, "K": K, "rmax": RMAX, "coeffs": c.tolist(), "lambdas": lam.tolist(),
               "max_rel_error": err}, open(OUT, "w"), indent=1)
    print("coeffs", c, "lambdas", lam, "max relative error", err)
