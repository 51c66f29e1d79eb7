"""Chain diagnostics of Sec. 3.1: integrated autocorrelation time (IAT),
effective sample size (ESS) and cost per effective sample (CES).

For a retained chain of N draws with IAT kappa that took T seconds,
    ESS = N / kappa,    CES = kappa T / N   (seconds per effective sample),
the definitions the paper uses to compare samplers (Table 1).  The paper does
not say how kappa is estimated; here it is Geyer's initial monotone sequence
estimator (Geyer 1992, "Practical Markov chain Monte Carlo", Stat. Sci. 7):
with sample autocorrelations r_t, the pair sums G_m = r_{2m} + r_{2m+1} are
summed while they stay positive, each capped by the previous one, and
    kappa = -1 + 2 sum_m G_m   ( = 1 + 2 sum_{t>=1} r_t for the kept lags).

Host-side numpy on traces the device chain records (gmrf_set_trace).
"""
from __future__ import annotations

import numpy as np


def autocorrelation(x) -> np.ndarray:
    """Sample autocorrelations r_0..r_{N-1} of a 1-D series:
    r_t = c_t / c_0 with c_t = (1/N) sum_{i<N-t} (x_i - xbar)(x_{i+t} - xbar),
    computed by FFT with zero padding (no circular wrap)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if n < 2:
        raise ValueError("autocorrelation needs at least 2 draws")
    d = x - x.mean()
    size = 1 << int(np.ceil(np.log2(2 * n)))
    f = np.fft.rfft(d, size)
    c = np.fft.irfft(f * np.conj(f), size)[:n] / n
    if c[0] <= 0.0:
        raise ValueError("autocorrelation of a constant series is undefined")
    return c / c[0]


def iat(x) -> float:
    """Integrated autocorrelation time by Geyer's initial monotone sequence."""
    r = autocorrelation(x)
    n = r.size
    total = 0.0
    prev = np.inf
    for m in range(n // 2):
        g = r[2 * m] + r[2 * m + 1]
        if g <= 0.0:
            break
        g = min(g, prev)
        total += g
        prev = g
    return max(-1.0 + 2.0 * total, 1.0 / n)


def ess(x) -> float:
    """Effective sample size N / IAT."""
    x = np.asarray(x, dtype=np.float64)
    return x.size / iat(x)


def ces(seconds: float, n_draws: int, kappa: float) -> float:
    """Cost per effective sample kappa T / N (seconds)."""
    return kappa * seconds / n_draws


def summary(x, seconds: float) -> dict:
    """IAT, ESS and CES of one retained chain that took `seconds`."""
    x = np.asarray(x, dtype=np.float64)
    k = iat(x)
    return {"n": int(x.size), "iat": k, "ess": x.size / k, "ces_s": ces(seconds, x.size, k),
            "seconds": float(seconds)}
