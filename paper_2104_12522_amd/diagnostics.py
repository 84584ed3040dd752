"""Sampler diagnostics for the chain histories a retrieval returns (host post-processing).

Sec. 5 and App. C: steps per effectively independent sample (SPEIS) from each chain's
autocorrelation, taken up to the first lag where it drops to a threshold (BART reports
the largest SPEIS over chains and parameters as a conservative value); effective sample
size ESS = kept steps / SPEIS; the Gelman & Rubin (1992) potential scale reduction; the
standard error of a posterior mean from ESS (App. C).
All functions take histories shaped [n_steps][n_chains][n_params], as Retrieval keeps
them, and vectorise over chains and parameters.
"""
from __future__ import annotations

import numpy as np


def autocorrelation(history: np.ndarray) -> np.ndarray:
    """Normalised autocorrelation rho[k][c][p] of every chain and parameter: the lag-k
    autocovariance with divisor n (Wiener-Khinchin: inverse transform of the power
    spectrum of the zero-padded, mean-removed series) over the lag-0 value."""
    h = np.asarray(history, dtype=np.float64)
    n = h.shape[0]
    x = h - h.mean(axis=0, keepdims=True)
    size = 1
    while size < 2 * n:
        size *= 2
    spec = np.fft.rfft(x, n=size, axis=0)
    acov = np.fft.irfft(spec.real ** 2 + spec.imag ** 2, n=size, axis=0)[:n] / n
    var = acov[0]
    safe = np.where(var > 0, var, 1.0)
    rho = acov / safe
    rho[:, var <= 0] = 0.0
    rho[0, var <= 0] = 1.0
    return rho


def speis_per_chain(history: np.ndarray, threshold: float = 0.01) -> np.ndarray:
    """SPEIS[c][p] = 1 + 2 sum_{k=1}^{K} rho_k, with K the last lag before rho first
    falls to or below the threshold."""
    rho = autocorrelation(history)
    below = rho[1:] <= threshold
    # first lag (1-based) at or below the threshold; n when it never gets there
    first = np.where(below.any(axis=0), below.argmax(axis=0) + 1, rho.shape[0])
    lags = np.arange(1, rho.shape[0])[:, None, None]
    keep = lags < first[None]
    return 1.0 + 2.0 * np.sum(np.where(keep, rho[1:], 0.0), axis=0)


def speis(history: np.ndarray, threshold: float = 0.01) -> float:
    """The conservative SPEIS: the largest over chains and parameters."""
    return float(speis_per_chain(history, threshold).max())


def ess(history: np.ndarray, threshold: float = 0.01) -> float:
    """Effective sample size: all kept steps of all chains over the conservative SPEIS."""
    h = np.asarray(history)
    return h.shape[0] * h.shape[1] / speis(h, threshold)


def ess_per_parameter(history: np.ndarray, threshold: float = 0.01) -> np.ndarray:
    """Per parameter: kept steps over that parameter's largest SPEIS across chains."""
    h = np.asarray(history)
    return h.shape[0] * h.shape[1] / speis_per_chain(h, threshold).max(axis=0)


def integrated_time_multichain(history: np.ndarray) -> np.ndarray:
    """Integrated autocorrelation time per parameter from all chains together (the
    within/between-chain method of Vehtari et al., the alternative to SPEIS that Sec. 5
    discusses): combined autocorrelation rho_t = 1 - (W - mean_c acov_c(t)) / var_plus,
    var_plus = (n-1)/n W + B/n, summed with Geyer's initial monotone sequence of pair
    sums. Unlike the largest per-chain SPEIS it includes the spread between chains, so
    it does not shrink when every chain is still far from independent samples."""
    h = np.asarray(history, dtype=np.float64)
    n, m, n_par = h.shape
    x = h - h.mean(axis=0, keepdims=True)
    size = 1
    while size < 2 * n:
        size *= 2
    out = np.empty(n_par)
    w = h.var(axis=0, ddof=1).mean(axis=0)
    b_over_n = h.mean(axis=0).var(axis=0, ddof=1)
    var_plus = (n - 1.0) / n * w + b_over_n
    for p in range(n_par):
        spec = np.fft.rfft(x[:, :, p], n=size, axis=0)
        acov = np.fft.irfft(spec.real ** 2 + spec.imag ** 2, n=size, axis=0)[:n] / n
        rho = 1.0 - (w[p] - acov.mean(axis=1)) / var_plus[p]
        pairs = rho[0:2 * (n // 2):2] + rho[1:2 * (n // 2):2]
        neg = np.flatnonzero(pairs < 0.0)
        pairs = pairs[:neg[0]] if neg.size else pairs
        out[p] = -1.0 + 2.0 * np.minimum.accumulate(pairs).sum()
    return out


def ess_multichain(history: np.ndarray) -> np.ndarray:
    """Per parameter: all kept steps of all chains over the multi-chain integrated time."""
    h = np.asarray(history)
    return h.shape[0] * h.shape[1] / integrated_time_multichain(h)


def gelman_rubin(history: np.ndarray) -> np.ndarray:
    """Potential scale reduction per parameter from m chains of n steps:
    sqrt(((n-1)/n W + (m+1)/(m n) B) / W), W the mean within-chain variance and B/n the
    variance of the chain means."""
    h = np.asarray(history, dtype=np.float64)
    n, m = h.shape[0], h.shape[1]
    chain_means = h.mean(axis=0)
    within = h.var(axis=0, ddof=1).mean(axis=0)
    between = n * chain_means.var(axis=0, ddof=1)
    pooled = (n - 1.0) / n * within + (m + 1.0) / (m * n) * between
    return np.sqrt(pooled / within)


def marginal_summary(history: np.ndarray):
    """Posterior mean and standard deviation per parameter over all kept states."""
    flat = np.asarray(history, dtype=np.float64).reshape(-1, np.shape(history)[-1])
    return flat.mean(axis=0), flat.std(axis=0)
