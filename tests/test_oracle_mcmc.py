"""Pins of the reference DE-MCz sampler: the random stream against published values, and
the sampler against targets whose posterior is known in closed form."""
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import mcmc


def test_splitmix64_reference_values(golden_dir):
    vals = [int(l) for l in open(os.path.join(golden_dir, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    assert [mcmc.splitmix64(1234567, k) for k in range(5)] == vals


def test_uniforms_and_normals():
    u = np.array([mcmc.u01(99, k) for k in range(20000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    z = np.array([mcmc.normal(7, g, c, 50, 0) for g in range(100) for c in range(50)])
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_proposal_uses_two_distinct_archive_rows():
    lo, hi = np.zeros(3), np.ones(3)
    x, z = mcmc.init_state(5, 40, 30, lo, hi)
    for g in range(30):
        y, r1, r2 = mcmc.propose(x, z, len(z), g, 5, lo, hi, 0.0)
        assert np.all(r1 != r2) and r1.min() >= 0 and r2.max() < len(z)
        gamma = 1.0 if g % 10 == 9 else 2.38 / math.sqrt(6.0)
        np.testing.assert_allclose(y, x + gamma * (z[r1] - z[r2]), rtol=0, atol=1e-15)


def _gauss_chi2(mu, cov):
    icov = np.linalg.inv(cov)

    def chi2(y):
        d = y - mu
        return np.einsum("ci,ij,cj->c", d, icov, d)
    return chi2


def test_gaussian_target_moments():
    # posterior N(mu, cov) well inside the prior box: sample mean and covariance
    mu = np.array([0.3, -0.2])
    cov = np.array([[0.04, 0.015], [0.015, 0.02]])
    lo, hi = np.full(2, -3.0), np.full(2, 3.0)
    hist, acc = mcmc.run(_gauss_chi2(mu, cov), 16, 3000, lo, hi, seed=11, thin=5)
    s = hist[500:].reshape(-1, 2)
    n_eff = s.shape[0] / 20.0           # conservative: correlated draws
    se = np.sqrt(np.diag(cov) / n_eff)
    assert np.all(np.abs(s.mean(0) - mu) < 5 * se)
    np.testing.assert_allclose(np.cov(s.T), cov, rtol=0.15, atol=0.003)
    assert 0.1 < acc.mean() / 3000 < 0.6


def test_flat_likelihood_samples_the_prior_box():
    lo, hi = np.array([-1.0, 2.0]), np.array([1.0, 5.0])
    hist, _ = mcmc.run(lambda y: np.zeros(len(y)), 16, 3000, lo, hi, seed=3, thin=5)
    s = hist[300::25].reshape(-1, 2)          # thinned: the KS test assumes independence
    for p in range(2):
        assert stats.kstest((s[:, p] - lo[p]) / (hi[p] - lo[p]), "uniform").pvalue > 1e-4


def test_delayed_acceptance_keeps_the_posterior():
    # a deliberately biased, miscalibrated surrogate: the two-stage chain still samples
    # the exact posterior, only with a lower acceptance rate
    mu = np.array([0.1, 0.4])
    cov = np.diag([0.03, 0.05])
    exact = _gauss_chi2(mu, cov)
    surr = _gauss_chi2(mu + np.array([0.1, -0.1]), cov * 1.8)
    lo, hi = np.full(2, -3.0), np.full(2, 3.0)
    hist, acc = mcmc.run(exact, 16, 3000, lo, hi, seed=21, thin=5, surrogate_chi2=surr)
    s = hist[500:].reshape(-1, 2)
    n_eff = s.shape[0] / 25.0
    se = np.sqrt(np.diag(cov) / n_eff)
    assert np.all(np.abs(s.mean(0) - mu) < 5 * se)
    np.testing.assert_allclose(np.diag(np.cov(s.T)), np.diag(cov), rtol=0.2)
