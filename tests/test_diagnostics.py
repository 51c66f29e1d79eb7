"""Pins for the chain diagnostics (Sec. 3.1: IAT, ESS = N / IAT,
CES = IAT T / N), each against something other than the code itself."""
import json
import os

import numpy as np
import pytest

from paper_1702_05518_amd import diagnostics as D

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_costs.json")


def test_autocorrelation_equals_its_definition():
    x = np.random.default_rng(0).normal(size=301).cumsum()
    n = x.size
    d = x - x.mean()
    c = np.array([np.dot(d[: n - t], d[t:]) / n for t in range(n)])
    assert np.allclose(D.autocorrelation(x), c / c[0], rtol=0, atol=1e-12)


@pytest.mark.parametrize("phi", [0.0, 0.5, 0.9])
def test_iat_of_ar1_matches_closed_form(phi):
    """x_t = phi x_{t-1} + e_t has r_t = phi^t, so IAT = (1 + phi) / (1 - phi)."""
    rng = np.random.default_rng(1)
    n = 400_000
    e = rng.normal(size=n)
    x = np.empty(n)
    x[0] = e[0] / np.sqrt(1 - phi * phi)
    for t in range(1, n):
        x[t] = phi * x[t - 1] + e[t]
    exact = (1 + phi) / (1 - phi)
    assert abs(D.iat(x) / exact - 1) < 0.08
    assert abs(D.ess(x) / (n / exact) - 1) < 0.08


def test_iat_of_two_site_gibbs_chain(orc):
    """A single edge: with tau, lam fixed the chromatic (= systematic) Gibbs
    chain of one coordinate is AR(1) with coefficient rho^2, where
    rho = tau / (tau + lam) is the posterior correlation of the two sites, so
    IAT = (1 + rho^2) / (1 - rho^2)."""
    rp = np.array([0, 1, 2], dtype=np.int64)
    cl = np.array([1, 0], dtype=np.int32)
    tau, lam = 2.0, 1.0
    ch = orc.Chain(rp, cl, np.array([0, 1], dtype=np.int32), np.array([0.3, -0.2]),
                   tau0=tau, lam0=lam, seed=4)
    n = 100_000
    x0 = np.empty(n)
    for t in range(n):
        ch.sweeps(1, hyper=False)
        x0[t] = ch.x[0]
    r2 = (tau / (tau + lam)) ** 2
    exact = (1 + r2) / (1 - r2)
    assert abs(D.iat(x0) / exact - 1) < 0.06


def test_table1_cost_arithmetic():
    """ESS = N / IAT and CES = IAT T / N reproduce Table 1 to its rounding."""
    g = json.load(open(GOLDEN))
    n = g["n_retained"]
    for row in g["rows"]:
        assert abs(n / row["ess"] - row["iat"]) <= 0.01, row
        assert round(D.ces(row["seconds"], n, n / row["ess"]), 2) == row["ces"], row
        assert abs(D.ces(row["seconds"], n, row["iat"]) - row["ces"]) <= 0.01, row
    chrom, block = g["rows"][0], g["rows"][1]
    # the stated improvement of the chromatic sampler's CES over block updating
    assert round(100 * (1 - chrom["ces"] / block["ces"])) == 89


def test_summary_and_errors():
    x = np.random.default_rng(3).normal(size=2000)
    s = D.summary(x, 10.0)
    assert s["n"] == 2000 and abs(s["ess"] * s["iat"] - 2000) < 1e-9
    assert abs(s["ces_s"] - s["iat"] * 10.0 / 2000) < 1e-15
    assert 0.8 < s["iat"] < 1.25            # white noise
    with pytest.raises(ValueError):
        D.iat(np.ones(10))
    with pytest.raises(ValueError):
        D.iat([1.0])
