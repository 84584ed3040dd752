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
