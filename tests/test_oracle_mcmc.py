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


def test_fixed_parameter_proposals():
    # a parameter with lo = hi: initial states and archive hold its value, no DE move or
    # jitter changes it, and gamma counts the two free parameters only
    lo, hi = np.zeros(3), np.ones(3)
    lo[1] = hi[1] = 0.25
    assert mcmc.free_count(lo, hi) == 2
    x, z = mcmc.init_state(5, 40, 30, lo, hi)
    assert np.all(x[:, 1] == 0.25) and np.all(z[:, 1] == 0.25)
    for g in range(12):
        y, r1, r2 = mcmc.propose(x, z, len(z), g, 5, lo, hi, 1e-6)
        assert np.all(y[:, 1] == 0.25)
        y0, r1, r2 = mcmc.propose(x, z, len(z), g, 5, lo, hi, 0.0)
        gamma = 1.0 if g % 10 == 9 else 2.38 / math.sqrt(4.0)
        np.testing.assert_allclose(y0, x + gamma * (z[r1] - z[r2]), rtol=0, atol=1e-15)


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


# ---- snooker moves (ter Braak & Vrugt 2008) ------------------------------------------
_MU4 = np.array([0.3, -0.2, 0.1, 0.0])
_COV4 = np.array([[1.0, 0.6, 0.0, 0.0], [0.6, 1.0, 0.3, 0.0],
                  [0.0, 0.3, 1.0, -0.4], [0.0, 0.0, -0.4, 1.0]]) * 0.04


def test_snooker_move_geometry():
    # the move stays on the line through x and z, and its length is gamma_s times the
    # orthogonal projection of z_R1 - z_R2 onto that line (least squares onto the line's
    # direction); the proposal factor is the (d-1)-th power of the distance ratio to z
    g = np.random.default_rng(4)
    for d in (2, 5, 9):
        x, zz, z1, z2 = g.normal(size=(4, d))
        y, log_q = mcmc.snooker(x, zz, z1, z2, 1.7)
        u = (x - zz)[:, None]
        coef, *_ = np.linalg.lstsq(u, z1 - z2, rcond=None)      # projection coefficient
        np.testing.assert_allclose(y - x, 1.7 * coef[0] * (x - zz), rtol=1e-12, atol=1e-14)
        _, res, *_ = np.linalg.lstsq(u, y - x, rcond=None)
        assert res.size == 0 or res[0] < 1e-24                   # collinear with x - z
        ratio = np.linalg.norm(y - zz) / np.linalg.norm(x - zz)
        assert log_q == pytest.approx((d - 1) * np.log(ratio), rel=1e-12, abs=1e-14)
    # x on the archive member: no line, no move
    y, log_q = mcmc.snooker(np.ones(3), np.ones(3), np.zeros(3), np.full(3, 2.0), 1.5)
    assert np.array_equal(y, np.ones(3)) and log_q == -np.inf


def test_snooker_third_row_is_uniform_over_the_others():
    for m, r1, r2 in ((3, 0, 2), (7, 2, 5), (7, 5, 2), (9, 3, 4), (5, 4, 0)):
        n = 6000
        rows = [mcmc.third_row((k + 0.5) / n, m, r1, r2) for k in range(n)]
        counts = np.bincount(rows, minlength=m)
        assert counts[r1] == 0 and counts[r2] == 0 and len(counts) == m
        others = [counts[i] for i in range(m) if i not in (r1, r2)]
        assert max(others) - min(others) <= 1


def test_snooker_moves_alone_sample_a_correlated_gaussian():
    # pure snooker (every move): a wrong proposal factor shifts these variances by
    # 25-60 %, outside the tolerance
    hist, acc = mcmc.run(_gauss_chi2(_MU4, _COV4), 16, 2500, np.full(4, -3.0), np.full(4, 3.0),
                         seed=7, thin=5, p_snooker=1.0)
    s = hist[500:].reshape(-1, 4)
    se = np.sqrt(np.diag(_COV4) / (s.shape[0] / 25.0))
    assert np.all(np.abs(s.mean(0) - _MU4) < 5 * se)
    np.testing.assert_allclose(s.var(0), np.diag(_COV4), rtol=0.15)
    assert 0.1 < acc.mean() / 2500 < 0.8


def test_fixed_parameters_with_snooker_moves_sample_the_conditional():
    # two of the four parameters held at their means (lo = hi): no move changes them, and
    # with snooker moves only the free pair samples the conditional Gaussian. The move's
    # proposal factor is a power of the distance ratio set by the dimension the chains move
    # in (2 here); taken over all four dimensions it nearly doubles these variances
    lo, hi = np.full(4, -3.0), np.full(4, 3.0)
    lo[2:] = hi[2:] = _MU4[2:]
    hist, acc = mcmc.run(_gauss_chi2(_MU4, _COV4), 16, 2500, lo, hi, seed=13, thin=5, p_snooker=1.0)
    assert np.all(hist[:, :, 2:] == _MU4[2:])
    s = hist[500:, :, :2].reshape(-1, 2)
    b = _COV4[:2, 2:]
    cond = _COV4[:2, :2] - b @ np.linalg.solve(_COV4[2:, 2:], b.T)
    se = np.sqrt(np.diag(cond) / (s.shape[0] / 25.0))
    assert np.all(np.abs(s.mean(0) - _MU4[:2]) < 5 * se)
    np.testing.assert_allclose(s.var(0), np.diag(cond), rtol=0.15)
    assert 0.1 < acc.mean() / 2500 < 0.9


def test_demczs_with_delayed_acceptance_keeps_the_posterior():
    # half the moves snooker, a biased surrogate in stage 1 (which carries the snooker
    # factor; dropping it there shrinks these variances by about 40 %)
    surr = _gauss_chi2(_MU4 + np.array([0.05, -0.05, 0.02, 0.0]), _COV4 * 1.5)
    hist, acc = mcmc.run(_gauss_chi2(_MU4, _COV4), 16, 3000, np.full(4, -3.0), np.full(4, 3.0),
                         seed=9, thin=5, surrogate_chi2=surr, p_snooker=0.5)
    s = hist[500:].reshape(-1, 4)
    se = np.sqrt(np.diag(_COV4) / (s.shape[0] / 25.0))
    assert np.all(np.abs(s.mean(0) - _MU4) < 5 * se)
    np.testing.assert_allclose(s.var(0), np.diag(_COV4), rtol=0.15)


def test_zero_snooker_rate_is_plain_demcz():
    g = np.random.default_rng(6)
    x, z = g.normal(size=(9, 3)), g.normal(size=(40, 3))
    lo, hi = np.full(3, -9.0), np.full(3, 9.0)
    y0, _, _ = mcmc.propose(x, z, 40, 3, 17, lo, hi, 1e-6)
    y1, lq = mcmc.propose_zs(x, z, 40, 3, 17, lo, hi, 1e-6, 0.0)
    assert np.array_equal(y0, y1) and np.all(lq == 0.0)
    y2, lq2 = mcmc.propose_zs(x, z, 40, 3, 17, lo, hi, 1e-6, 0.5)
    moved = lq2 != 0.0
    assert 0 < moved.sum() < 9 and np.array_equal(y2[~moved], y0[~moved])
