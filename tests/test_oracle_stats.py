"""Pins of the sampler diagnostics against the paper's printed numbers (Table 4, App. C)."""
import os

import numpy as np
import pytest

from oracle import stats


def _rows(path):
    with open(path) as f:
        return [l.split() for l in f if l.strip() and not l.startswith("#")]


def test_table4_credible_region_errors(golden_dir):
    # every row and column of Table 4: s_C = sqrt(C (1 - C) / (ESS + 3)), in percent,
    # rounded to two decimals as printed
    rows = _rows(os.path.join(golden_dir, "table4_credible_region_error.txt"))
    assert len(rows) == 13
    for name, geom, speis, ess, *s in rows:
        for c, printed in zip((0.6827, 0.9545, 0.9973), s):
            got = 100 * stats.credible_region_error(c, float(ess))
            assert round(got, 2) == pytest.approx(float(printed), abs=1e-9), (name, geom, c)


def test_appendix_c_sample_sizes(golden_dir):
    for c, s, quoted in _rows(os.path.join(golden_dir, "appC_sample_sizes.txt")):
        n = stats.required_samples(float(c), float(s))
        assert abs(n - float(quoted)) / float(quoted) < 0.1


def test_sec5_iteration_budget():
    # Sec. 5: a 95.45 % region with ESS ~ 1700 has a 0.5 % uncertainty; SPEIS 1000
    # then needs 1.7e6 iterations
    assert stats.credible_region_error(0.9545, 1700) == pytest.approx(0.005, rel=0.02)


def test_speis_of_independent_samples_is_one():
    x = np.random.default_rng(0).normal(size=(4, 20000, 2))
    assert stats.speis(x, threshold=0.05) < 1.1


def test_speis_of_ar1_matches_integrated_autocorrelation():
    # AR(1) with coefficient a: integrated autocorrelation time (1 + a) / (1 - a)
    a = 0.8
    g = np.random.default_rng(1)
    n = 400_000
    eps = g.normal(size=n)
    x = np.empty(n)
    x[0] = eps[0]
    for i in range(1, n):
        x[i] = a * x[i - 1] + eps[i]
    s = stats.speis_chain(x, threshold=0.01)
    # truncation at rho <= 0.01 drops sum_{k>K} rho_k ~ 2 * 0.01 * a / (1 - a)
    assert s == pytest.approx((1 + a) / (1 - a), rel=0.06)


def test_gelman_rubin():
    g = np.random.default_rng(2)
    same = g.normal(size=(5, 5000, 3))
    assert np.all(np.abs(stats.gelman_rubin(same) - 1.0) < 0.01)
    shifted = same + np.arange(5)[:, None, None]
    assert np.all(stats.gelman_rubin(shifted) > 1.5)


def test_product_diagnostics_match_oracle():
    # the package's vectorised diagnostics against the oracle's per-chain definitions
    from paper_2104_12522_amd import diagnostics as dg
    g = np.random.default_rng(21)
    n, m, d = 400, 5, 3
    hist = np.empty((n, m, d))
    x = g.normal(size=(m, d))
    phi = np.array([0.0, 0.6, 0.95])
    for t in range(n):
        x = phi * x + np.sqrt(1 - phi ** 2) * g.normal(size=(m, d))
        hist[t] = x
    chains = hist.transpose(1, 0, 2)           # oracle layout [chain][step][param]
    for c in range(m):
        for p in range(d):
            assert dg.speis_per_chain(hist)[c, p] == pytest.approx(
                stats.speis_chain(chains[c, :, p]), rel=1e-10)
    assert dg.speis(hist) == pytest.approx(stats.speis(chains), rel=1e-10)
    assert dg.ess(hist) == pytest.approx(stats.ess(chains), rel=1e-10)
    np.testing.assert_allclose(dg.gelman_rubin(hist), stats.gelman_rubin(chains), rtol=1e-12)


def _ar1_chains(a, m, n, seed):
    g = np.random.default_rng(seed)
    x = np.empty((m, n))
    x[:, 0] = g.normal(size=m) / np.sqrt(1 - a * a)      # stationary start
    eps = g.normal(size=(m, n))
    for i in range(1, n):
        x[:, i] = a * x[:, i - 1] + eps[:, i]
    return x


def test_multichain_time_of_ar1_matches_closed_form():
    # AR(1) chains with coefficient a: tau = (1 + a) / (1 - a); the estimator's error on
    # m chains of n steps is of order tau sqrt(tau / (m n))
    for a in (0.5, 0.9):
        x = _ar1_chains(a, 8, 40_000, seed=int(a * 10))
        tau = stats.integrated_time_multichain(x[:, :, None])[0]
        assert tau == pytest.approx((1 + a) / (1 - a), rel=0.08)
    # independent samples: tau ~ 1
    x = np.random.default_rng(5).normal(size=(6, 20_000, 1))
    assert stats.integrated_time_multichain(x)[0] == pytest.approx(1.0, abs=0.06)


def test_multichain_time_counts_chains_that_have_not_mixed():
    # chains that each sit at their own level (no mixing between them within the run):
    # per-chain autocorrelations look independent, the combined estimate does not
    g = np.random.default_rng(6)
    x = g.normal(size=(8, 5000, 1)) + 3.0 * g.normal(size=(8, 1, 1))
    assert stats.speis(x, threshold=0.01) < 1.5
    assert stats.integrated_time_multichain(x)[0] > 100


def test_product_multichain_time_matches_oracle():
    from paper_2104_12522_amd import diagnostics as dg
    x = np.stack([_ar1_chains(a, 5, 3000, seed=9 + i) for i, a in enumerate((0.0, 0.7, 0.97))], axis=2)
    ref = stats.integrated_time_multichain(x)
    got = dg.integrated_time_multichain(x.transpose(1, 0, 2))
    np.testing.assert_allclose(got, ref, rtol=1e-9)
