"""Sampler diagnostics (oracle; test infrastructure only).

Sec. 5 and App. C: steps per effectively independent sample (SPEIS) from the
autocorrelation function, effective sample size (ESS), the standard errors of a
posterior mean, standard deviation and credible-region probability content, and the
Gelman-Rubin convergence statistic.
"""
from __future__ import annotations

import numpy as np


def autocorrelation(x: np.ndarray) -> np.ndarray:
    """Normalised autocorrelation function rho_k, k = 0..n-1, of one chain (FFT-based,
    biased estimator: lag-k autocovariance divided by n)."""
    x = np.asarray(x, dtype=np.float64) - np.mean(x)
    n = x.size
    m = 1 << int(np.ceil(np.log2(2 * n)))
    fx = np.fft.rfft(x, m)
    acov = np.fft.irfft(fx * np.conj(fx), m)[:n] / n
    if acov[0] == 0.0:
        out = np.zeros(n)
        out[0] = 1.0
        return out
    return acov / acov[0]


def speis_chain(x: np.ndarray, threshold: float = 0.01) -> float:
    """SPEIS of one parameter of one chain: the autocorrelation summed from lag 0 up to
    the lag where it first falls to the threshold, counted on both sides of lag 0:
    SPEIS = 1 + 2 sum_{k=1}^{K} rho_k, K = last lag before rho_k <= threshold."""
    rho = autocorrelation(x)
    total = 1.0
    for k in range(1, rho.size):
        if rho[k] <= threshold:
            break
        total += 2.0 * rho[k]
    return total


def speis(chains: np.ndarray, threshold: float = 0.01) -> float:
    """The largest SPEIS over all chains and parameters (Sec. 5, Sec. 6.3).
    chains: [n_chains][n_steps][n_params]."""
    c = np.asarray(chains, dtype=np.float64)
    return max(speis_chain(c[i, :, p], threshold)
               for i in range(c.shape[0]) for p in range(c.shape[2]))


def ess(chains: np.ndarray, threshold: float = 0.01) -> float:
    """ESS = total kept steps / SPEIS (Sec. 5)."""
    c = np.asarray(chains)
    return c.shape[0] * c.shape[1] / speis(c, threshold)


def integrated_time_multichain(chains: np.ndarray) -> np.ndarray:
    """Integrated autocorrelation time per parameter from m chains together (the
    within/between-chain method of Vehtari et al., which Sec. 5 discusses as the
    alternative to its SPEIS): the combined autocorrelation
    rho_t = 1 - (W - mean_c acov_c(t)) / var_plus, var_plus = (n-1)/n W + B/n,
    summed with Geyer's (1992) initial monotone sequence: pairs P_k = rho_2k + rho_2k+1
    while positive, made non-increasing, tau = -1 + 2 sum_k P_k.
    chains: [m][n][n_params]. ESS = m n / tau."""
    c = np.asarray(chains, dtype=np.float64)
    m, n, n_par = c.shape
    out = np.empty(n_par)
    for p in range(n_par):
        acov = np.array([autocorrelation(c[i, :, p]) * np.var(c[i, :, p]) for i in range(m)])
        w = np.mean([np.var(c[i, :, p], ddof=1) for i in range(m)])
        b_over_n = np.var([np.mean(c[i, :, p]) for i in range(m)], ddof=1)
        var_plus = (n - 1.0) / n * w + b_over_n
        rho = 1.0 - (w - acov.mean(axis=0)) / var_plus
        total, prev = 0.0, np.inf
        for k in range(n // 2):
            pair = rho[2 * k] + rho[2 * k + 1]
            if pair < 0.0:
                break
            prev = min(prev, pair)
            total += prev
        out[p] = -1.0 + 2.0 * total
    return out


def credible_region_error(c_hat: float, n: float) -> float:
    """Posterior standard deviation of the probability content of a credible region
    from n independent samples (App. C): s_C = sqrt(C (1 - C) / (n + 3))."""
    return float(np.sqrt(c_hat * (1.0 - c_hat) / (n + 3.0)))


def required_samples(c_hat: float, s_c: float) -> float:
    """Eq. 1 / App. C: N ~ C (1 - C) / s_C^2."""
    return c_hat * (1.0 - c_hat) / s_c ** 2


def mean_standard_error(sigma_hat: float, n: float) -> float:
    """App. C: s_mu = sigma_hat / sqrt(N)."""
    return sigma_hat / np.sqrt(n)


def sigma_relative_error(n: float) -> float:
    """App. C: s_sigma / sigma ~ sqrt(1 / (2N))."""
    return float(np.sqrt(1.0 / (2.0 * n)))


def gelman_rubin(chains: np.ndarray) -> np.ndarray:
    """Gelman & Rubin (1992) potential scale reduction per parameter:
    W = mean within-chain variance, B/n = variance of the chain means,
    V = (n-1)/n W + (m+1)/(m n) B,  R = sqrt(V / W).
    chains: [m][n][n_params]."""
    c = np.asarray(chains, dtype=np.float64)
    m, n = c.shape[0], c.shape[1]
    means = c.mean(axis=1)
    w = c.var(axis=1, ddof=1).mean(axis=0)
    b = n * means.var(axis=0, ddof=1)
    v = (n - 1.0) / n * w + (m + 1.0) / (m * n) * b
    return np.sqrt(v / w)
