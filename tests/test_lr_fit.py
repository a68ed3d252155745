"""The long-range Ising input (tests/golden/lr_fit_K6.json, written by tests/golden/make_lr_fit.py):
J(r) = r^-2 on r = 1..99 as six exponentials. Pinned to the function it approximates and to a fresh
run of the fitting script."""
import importlib.util
import json
import os

import numpy as np

HERE = os.path.join(os.path.dirname(__file__), "golden")


def test_fit_reproduces_power_law_and_script():
    fit = json.load(open(os.path.join(HERE, "lr_fit_K6.json")))
    c, lam = np.array(fit["coeffs"]), np.array(fit["lambdas"])
    assert len(c) == len(lam) == 6
    assert np.all((lam > 0) & (lam < 1)) and np.all(c > 0)   # a completely monotone target
    r = np.arange(1, 100)
    J = (c[None, :] * lam[None, :] ** (r[:, None] - 1)).sum(1)
    rel = np.abs(J - r ** -2.0) / r ** -2.0
    assert rel[:10].max() < 1e-3 and rel.max() < 0.05
    assert abs(rel.max() - fit["max_rel_error"]) < 1e-12
    spec = importlib.util.spec_from_file_location("make_lr_fit", os.path.join(HERE, "make_lr_fit.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    c2, lam2, _ = mod.fit()
    assert np.allclose(c2, c, rtol=1e-9) and np.allclose(lam2, lam, rtol=1e-9)
