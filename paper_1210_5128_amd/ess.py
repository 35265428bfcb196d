"""Effective sample size and convergence diagnostics of MCMC traces
(host-side reporting).

Geyer's initial monotone sequence estimator (Geyer, "Practical Markov chain
Monte Carlo", Statistical Science 1992): autocorrelations rho_k of one chain's
trace, pair sums G_m = rho_{2m} + rho_{2m+1}, truncated at the first
non-positive pair and made non-increasing; tau = -1 + 2 sum_m G_m and
ESS = N / tau.  ``ess`` sums the per-chain ESS.

Several chains together (Vehtari, Gelman, Simpson, Carpenter, Buerkner,
"Rank-normalization, folding, and localization: an improved R-hat", Bayesian
Analysis 2021): ``ess_multichain`` takes the autocorrelations from the
within-chain autocovariances against the pooled variance estimate
var+ = (N-1)/N W + B/N, so chains that disagree (B >> W) give a small ESS;
``ess_bulk`` applies it to the rank-normalised split chains, and
``rhat_rank`` is the larger of the rank-normalised split-R-hat and that of the
folded draws |x - median|.
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


def _burned(traces: np.ndarray, burn: float) -> np.ndarray:
    traces = np.atleast_2d(np.asarray(traces, dtype=np.float64))
    return traces[:, int(burn * traces.shape[1]):]


def _split(x: np.ndarray) -> np.ndarray:
    """Each chain [C][T] cut into its two halves: [2C][T // 2]."""
    h = x.shape[1] // 2
    return np.concatenate([x[:, :h], x[:, h:2 * h]], axis=0)


def _rhat_plain(x: np.ndarray) -> float:
    m, n = x.shape
    if n < 2:
        return float("nan")
    W = x.var(axis=1, ddof=1).mean()
    if W == 0:
        return 1.0 if np.all(x == x.flat[0]) else float("inf")
    B = n * x.mean(axis=1).var(ddof=1) if m > 1 else 0.0
    return float(np.sqrt(((n - 1) / n * W + B / n) / W))


def rank_normalize(x: np.ndarray) -> np.ndarray:
    """Pooled ranks r (ties averaged) -> normal scores ndtri((r - 3/8) / (S + 1/4))."""
    from scipy.special import ndtri
    from scipy.stats import rankdata
    r = rankdata(x, method="average").reshape(x.shape)
    return ndtri((r - 0.375) / (x.size + 0.25))


def ess_multichain(x: np.ndarray) -> float:
    """ESS of M chains [M][N] together (no burn-in handling; see ess_bulk)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    M, N = x.shape
    if N < 4:
        return float(M * N)
    if np.all(x == x.flat[0]):
        return 1.0
    xc = x - x.mean(axis=1, keepdims=True)
    f = np.fft.rfft(xc, n=2 * N, axis=1)
    acov = np.fft.irfft(f * np.conj(f), axis=1)[:, :N] / N        # biased autocovariance per chain
    W = x.var(axis=1, ddof=1).mean()
    var_plus = (N - 1) / N * W + (x.mean(axis=1).var(ddof=1) if M > 1 else 0.0)
    if var_plus <= 0:
        return float(M * N)
    rho = 1.0 - (W - acov.mean(axis=0)) / var_plus
    rho[0] = 1.0
    tau = -1.0
    prev = np.inf
    for m in range(N // 2):
        g = rho[2 * m] + rho[2 * m + 1]
        if g <= 0:
            break
        g = min(g, prev)
        tau += 2.0 * g
        prev = g
    tau = max(tau, 1.0 / (M * N))
    return float(M * N / tau)


def ess_bulk(traces: np.ndarray, burn: float = 0.2) -> float:
    """Rank-normalised multi-chain ESS of the split chains after burn-in."""
    x = _burned(traces, burn)
    if x.shape[1] < 8:
        return float("nan")
    return ess_multichain(rank_normalize(_split(x)))


def rhat_rank(traces: np.ndarray, burn: float = 0.2) -> float:
    """Rank-normalised split-R-hat: max over the draws and the folded draws."""
    x = _burned(traces, burn)
    if x.shape[1] < 4:
        return float("nan")
    z = _split(x)
    folded = np.abs(z - np.median(z))
    return max(_rhat_plain(rank_normalize(z)), _rhat_plain(rank_normalize(folded)))


def mcse_mean(traces: np.ndarray, burn: float = 0.2) -> float:
    """Monte Carlo standard error of the pooled mean after burn-in: sd / sqrt(multi-chain ESS)."""
    x = _burned(traces, burn)
    e = ess_multichain(_split(x)) if x.shape[1] >= 8 else float(x.size)
    return float(x.std(ddof=1) / np.sqrt(max(e, 1.0))) if x.size > 1 else float("nan")


def agree_within_mcse(a: np.ndarray, b: np.ndarray, burn: float = 0.2, k: float = 3.0):
    """Whether the pooled means of two samplers' traces agree within k combined MCSE:
    returns (|mean_a - mean_b|, k * sqrt(mcse_a^2 + mcse_b^2), agree)."""
    xa, xb = _burned(a, burn), _burned(b, burn)
    d = abs(float(xa.mean()) - float(xb.mean()))
    tol = k * float(np.hypot(mcse_mean(a, burn), mcse_mean(b, burn)))
    return d, tol, bool(d <= tol)
