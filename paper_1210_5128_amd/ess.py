"""Effective sample size of MCMC traces (host-side reporting).

Geyer's initial monotone sequence estimator (Geyer, "Practical Markov chain
Monte Carlo", Statistical Science 1992): autocorrelations rho_k of one chain's
trace, pair sums G_m = rho_{2m} + rho_{2m+1}, truncated at the first
non-positive pair and made non-increasing; tau = -1 + 2 sum_m G_m and
ESS = N / tau.  Several chains: the sum of the per-chain ESS.
"""
from __future__ import annotations

import numpy as np


def autocorr(x: np.ndarray) -> np.ndarray:
    """Normalised autocorrelation of a 1-D trace (FFT, biased estimator)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    x = x - x.mean()
    f = np.fft.rfft(x, n=2 * n)
    ac = np.fft.irfft(f * np.conj(f))[:n]
    if ac[0] <= 0:
        return np.concatenate([[1.0], np.zeros(n - 1)])
    return ac / ac[0]


def ess_chain(x: np.ndarray) -> float:
    """ESS of one chain (a constant trace has ESS 1)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if n < 4 or np.all(x == x[0]):
        return 1.0 if n else 0.0
    rho = autocorr(x)
    tau = -1.0
    prev = np.inf
    for m in range(n // 2):
        g = rho[2 * m] + rho[2 * m + 1]
        if g <= 0:
            break
        g = min(g, prev)
        tau += 2.0 * g
        prev = g
    tau = max(tau, 1.0 / n)
    return float(n / tau)


def ess(traces: np.ndarray, burn: float = 0.2) -> float:
    """Summed ESS over chains of traces [C][T] after dropping the first `burn` fraction."""
    traces = np.atleast_2d(np.asarray(traces, dtype=np.float64))
    start = int(burn * traces.shape[1])
    return float(sum(ess_chain(row[start:]) for row in traces))


def split_rhat(traces: np.ndarray, burn: float = 0.2) -> float:
    """Split-R-hat (Gelman et al.) of traces [C][T] after burn-in."""
    traces = np.atleast_2d(np.asarray(traces, dtype=np.float64))
    x = traces[:, int(burn * traces.shape[1]):]
    h = x.shape[1] // 2
    if h < 2:
        return float("nan")
    halves = np.concatenate([x[:, :h], x[:, h:2 * h]], axis=0)
    m, n = halves.shape
    means = halves.mean(axis=1)
    W = halves.var(axis=1, ddof=1).mean()
    B = n * means.var(ddof=1)
    if W == 0:
        return 1.0
    var = (n - 1) / n * W + B / n
    return float(np.sqrt(var / W))
