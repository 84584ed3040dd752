"""Pins of the oracle's line-shape and opacity arithmetic (Sec. 6.1.1, Eqs. 2-11)."""
import math

import numpy as np
import pytest
from scipy import integrate, optimize

from oracle import opacity as op
from workloads import LineList


def test_voigt_gaussian_limit():
    # gamma -> 0: V -> G (Eq. 2)
    sig = 0.013
    x = np.linspace(-5 * sig, 5 * sig, 101)
    v = op.voigt(x, sig, 1e-12 * sig)
    g = op.gaussian(x, sig)
    assert np.max(np.abs(v - g) / g) < 1e-8


def test_voigt_lorentzian_limit():
    # sigma -> 0: V -> L (Eq. 3)
    gam = 0.07
    x = np.linspace(-20 * gam, 20 * gam, 101)
    v = op.voigt(x, 1e-9 * gam, gam)
    lz = op.lorentzian(x, gam)
    assert np.max(np.abs(v - lz) / lz) < 1e-8


@pytest.mark.parametrize("sig,gam,x", [(0.01, 0.002, 0.0), (0.01, 0.02, 0.013),
                                       (0.03, 0.01, -0.09), (0.005, 0.05, 0.4)])
def test_voigt_is_the_convolution(sig, gam, x):
    # Eq. 10: V(nu) = int G(nu') L(nu - nu') dnu', evaluated by adaptive quadrature
    f = lambda t: op.gaussian(t, sig) * op.lorentzian(x - t, gam)
    val, _ = integrate.quad(f, -40 * sig, 40 * sig, points=[0.0, x], epsabs=0, epsrel=1e-12,
                            limit=500)
    assert op.voigt(np.array([x]), sig, gam)[0] == pytest.approx(val, rel=1e-9)


def test_voigt_unit_area():
    # the profile is normalised; the Lorentz tails beyond +-X carry 1 - (2/pi) atan(X/gamma)
    sig, gam = 0.02, 0.01
    X = 400.0
    x = np.linspace(-X, X, 4_000_001)
    area = np.trapezoid(op.voigt(x, sig, gam), x)
    tail = 1.0 - 2.0 / math.pi * math.atan(X / gam)
    assert area + tail == pytest.approx(1.0, abs=2e-7)


@pytest.mark.parametrize("sig,gam", [(0.01, 0.0), (0.0, 0.05), (0.01, 0.01), (0.003, 0.03)])
def test_voigt_hwhm_olivero(sig, gam):
    # Olivero & Longbothum (1977) quote ~0.02 % accuracy against the true Voigt HWHM
    hw = op.voigt_hwhm(sig, gam)
    if gam == 0.0:
        true = math.sqrt(2 * math.log(2)) * sig
    elif sig == 0.0:
        true = gam
    else:
        peak = op.voigt(np.array([0.0]), sig, gam)[0]
        true = optimize.brentq(lambda x: op.voigt(np.array([x]), sig, gam)[0] - peak / 2,
                               1e-9, 10 * (sig + gam), xtol=1e-15)
    assert hw == pytest.approx(true, rel=2.5e-4)


def test_line_strength_reference_temperature():
    s = op.line_strength(np.array([1e-21]), np.array([2000.0]), np.array([1500.0]), 296.0)
    assert s[0] == pytest.approx(1e-21, rel=1e-15)


def test_line_strength_boltzmann_ratio():
    # with nu0 large the stimulated-emission factor is ~1; ratio of two lines at the same
    # nu0 differing in E'' by dE follows exp(-c2 dE (1/T - 1/296))
    T = 1500.0
    s = op.line_strength(np.array([1.0, 1.0]), np.array([4000.0, 4000.0]),
                         np.array([0.0, 1000.0]), T)
    assert s[1] / s[0] == pytest.approx(math.exp(-1.4387769 * 1000.0 * (1 / T - 1 / 296.0)),
                                        rel=1e-13)


def test_widths_reference_conditions():
    assert op.lorentz_gamma(0.07, 296.0, 1.01325) == pytest.approx(0.07, rel=1e-15)
    # textbook Doppler half width: HWHM = 3.581e-7 nu0 sqrt(T / M[amu])
    sig = op.doppler_sigma(2000.0, 18.0, 296.0)
    hw = math.sqrt(2 * math.log(2)) * sig
    assert hw == pytest.approx(3.581e-7 * 2000.0 * math.sqrt(296.0 / 18.0), rel=2e-4)


def test_line_strength_partition_direction():
    # E'' = 0 removes the Boltzmann factor, and at nu0 = 1e5 cm^-1 the stimulated-emission
    # factor 1 - exp(-c2 nu0 / T) is 1 to within exp(-48) for every T below 3000 K, so
    # S(T)/S(296) is the partition ratio alone: Q ~ T^1.5 makes it (296/T)^1.5 -- a smaller
    # strength when hotter (Q(T)/Q(296) in its place would give the inverse)
    for T in (148.0, 592.0, 1184.0, 2960.0):
        s = op.line_strength(np.array([1.0]), np.array([1e5]), np.array([0.0]), T)[0]
        assert s == pytest.approx((296.0 / T) ** 1.5, rel=1e-12)
    # and between two temperatures S(T1)/S(T2) = (T2/T1)^1.5
    s1 = op.line_strength(np.array([1.0]), np.array([1e5]), np.array([0.0]), 700.0)[0]
    s2 = op.line_strength(np.array([1.0]), np.array([1e5]), np.array([0.0]), 2100.0)[0]
    assert s1 / s2 == pytest.approx(3.0 ** 1.5, rel=1e-12)


def test_line_strength_stimulated_emission_limit():
    # c2 nu0 << T: 1 - exp(-c2 nu0 / T) -> c2 nu0 / T, so the stimulated-emission factor
    # contributes 296/T and with the partition ratio S(T)/S(296) -> (296/T)^2.5; at
    # nu0 = 1e-4 cm^-1 the next order is c2 nu0 / (2 T) < 3e-7 relative
    for T in (1184.0, 2960.0):
        s = op.line_strength(np.array([1.0]), np.array([1e-4]), np.array([0.0]), T)[0]
        assert s == pytest.approx((296.0 / T) ** 2.5, rel=1e-6)
    # the factor is absent at the reference temperature whatever nu0
    s = op.line_strength(np.array([1.0, 1.0]), np.array([1e-4, 1e5]), np.array([0.0, 0.0]), 296.0)
    np.testing.assert_allclose(s, 1.0, rtol=1e-12)


def test_lorentz_width_scaling():
    # Eq. 3 widths scale linearly with pressure (in atmospheres) and as T^-1/2:
    # twice the pressure doubles the width, four times the reference temperature halves it
    g = 0.07
    assert op.lorentz_gamma(g, 296.0, 2 * 1.01325) == pytest.approx(2 * g, rel=1e-15)
    assert op.lorentz_gamma(g, 4 * 296.0, 1.01325) == pytest.approx(g / 2, rel=1e-15)
    assert op.lorentz_gamma(g, 4 * 296.0, 2 * 1.01325) == pytest.approx(g, rel=1e-15)
    # 1 bar is 1/1.01325 atm
    assert op.lorentz_gamma(g, 296.0, 1.0) == pytest.approx(g / 1.01325, rel=1e-15)


def test_doppler_width_scaling():
    # thermal Doppler width ~ nu0 sqrt(T / m): doubles at four times the temperature,
    # halves at four times the mass, doubles at twice the line centre
    base = op.doppler_sigma(2000.0, 18.0, 296.0)
    assert op.doppler_sigma(2000.0, 18.0, 4 * 296.0) == pytest.approx(2 * base, rel=1e-15)
    assert op.doppler_sigma(2000.0, 72.0, 296.0) == pytest.approx(base / 2, rel=1e-15)
    assert op.doppler_sigma(4000.0, 18.0, 296.0) == pytest.approx(2 * base, rel=1e-15)
    # absolute value at 1184 K: the textbook HWHM 3.581e-7 nu0 sqrt(T / M[amu])
    hw = math.sqrt(2 * math.log(2)) * op.doppler_sigma(3000.0, 44.0, 1184.0)
    assert hw == pytest.approx(3.581e-7 * 3000.0 * math.sqrt(1184.0 / 44.0), rel=2e-4)


def _single_line(nu0=2000.1, s=1e-20, g=0.07, e=300.0, m=18.015):
    return LineList(np.array([nu0]), np.array([s]), np.array([g]), np.array([e]),
                    np.array([m]))


def test_single_line_cell_is_strength_times_profile():
    # f01oneline idea (Table 1): a one-line table equals S(T) V(nu - nu0) inside the window
    ln = _single_line()
    T, p = 1442.58, 0.33516          # the f04broadening layer (Sec. 6.1.1)
    nu_start, dnu, n = 1990.0, 0.005, 4001
    cell = op.cell_cross_section(ln, T, p, nu_start, dnu, n)
    nu = nu_start + dnu * np.arange(n)
    s_t = op.line_strength(ln.s296, ln.nu0, ln.elow, T)[0]
    sig = op.doppler_sigma(ln.nu0, ln.mass_amu, T)[0]
    gam = op.lorentz_gamma(ln.gamma296, T, p)[0]
    hw = op.voigt_hwhm(sig, gam)
    inside = np.abs(nu - ln.nu0[0]) <= 25 * hw
    # reference from the convolution integral at a few points
    for k in np.flatnonzero(inside)[:: max(1, inside.sum() // 7)]:
        x = nu[k] - ln.nu0[0]
        f = lambda t: op.gaussian(t, sig) * op.lorentzian(x - t, gam)
        val, _ = integrate.quad(f, -40 * sig, 40 * sig, points=[0.0, x], epsabs=0,
                                epsrel=1e-12, limit=500)
        assert cell[k] == pytest.approx(s_t * val, rel=1e-8)
    assert np.all(cell[~inside] == 0.0)
    assert np.all(cell[inside] > 0.0)


def test_two_lines_add():
    # f06blending idea (Table 1): two lines ~0.04 cm^-1 apart sampled every 0.005 cm^-1
    a = _single_line(nu0=2000.00)
    b = _single_line(nu0=2000.04, s=3e-21, e=900.0)
    both = LineList(*(np.concatenate([getattr(a, f), getattr(b, f)])
                      for f in ("nu0", "s296", "gamma296", "elow", "mass_amu")))
    args = (1000.0, 0.01, 1999.5, 0.005, 201)
    ca = op.cell_cross_section(a, *args)
    cb = op.cell_cross_section(b, *args)
    cab = op.cell_cross_section(both, *args)
    np.testing.assert_allclose(cab, ca + cb, rtol=1e-14, atol=0)


def test_sampled_line_area_matches_truncated_profile():
    # a Lorentz-dominated line on a fine grid integrates to S times the profile mass
    # inside +-25 HWHM, which for a Lorentzian is (2/pi) atan(25 HWHM / gamma)
    ln = _single_line(g=0.08)
    T, p = 1000.0, 50.0
    nu_start, dnu, n = 1800.0, 0.002, 200_001
    cell = op.cell_cross_section(ln, T, p, nu_start, dnu, n)
    s_t = op.line_strength(ln.s296, ln.nu0, ln.elow, T)[0]
    sig = op.doppler_sigma(ln.nu0, ln.mass_amu, T)[0]
    gam = op.lorentz_gamma(ln.gamma296, T, p)[0]
    hw = op.voigt_hwhm(sig, gam)
    expected = s_t * 2.0 / math.pi * math.atan(25 * hw / gam)
    assert cell.sum() * dnu == pytest.approx(expected, rel=2e-4)


def test_cell_matches_pointwise_sum():
    # brute force point by point over a tiny random list equals the chunked cell routine
    g = np.random.default_rng(7)
    n = 40
    ln = LineList(g.uniform(2000, 2010, n), 10 ** g.uniform(-25, -19, n),
                  g.uniform(0.05, 0.1, n), g.uniform(0, 5000, n), g.uniform(18, 44, n))
    T, p = 1700.0, 3.0
    nu_start, dnu, nn = 1995.0, 0.05, 401
    cell = op.cell_cross_section(ln, T, p, nu_start, dnu, nn, chunk=7)
    for k in range(0, nn, 13):
        assert cell[k] == pytest.approx(op.point_cross_section(ln, T, p, nu_start + dnu * k),
                                        rel=1e-12, abs=1e-300)


# ---- profile-table mode (Sec. 4 items 4-6) ---------------------------------------------
F04_T, F04_P = 1442.58, 0.33516      # the f04broadening layer (Sec. 6.1.1)


def _widths(ln, T=F04_T, p=F04_P):
    s_t, sig, gam = op.table_line_parameters(ln, T, p)
    return float(s_t[0]), float(sig[0]), float(gam[0])


def test_table_mode_line_on_node_and_sample_equals_direct():
    # a line whose widths are grid nodes and whose centre is a fine sample: the table
    # mode samples the direct-mode profile (the two offsets differ by rounding only)
    ln = _single_line(nu0=2000.1)
    _, sig, gam = _widths(ln)
    tab = op.profile_table([sig / 2, sig, 2 * sig], [gam / 3, gam, 3 * gam], 0.005, 100, 25.0)
    nu_start, n = 1990.0, 4001
    got = op.table_cell_cross_section(ln, F04_T, F04_P, nu_start, n, tab)
    ref = op.cell_cross_section(ln, F04_T, F04_P, nu_start, 0.005, n)
    t_max = int(tab["ext"][1, 1])
    s = int(np.rint((ln.nu0[0] - nu_start) / tab["delta"]))
    t = np.arange(n) * 100 - s
    core = np.abs(t) < t_max - 100
    np.testing.assert_allclose(got[core], ref[core], rtol=1e-9)
    assert np.all(got[np.abs(t) > t_max] == 0.0) and np.all(got[np.abs(t) <= t_max] > 0.0)


def test_table_mode_translates_by_whole_output_intervals():
    # moving the centre by one output interval moves the sampled profile by one point
    a, b = _single_line(nu0=2000.1), _single_line(nu0=2000.105)
    _, sig, gam = _widths(a)
    tab = op.profile_table([sig], [gam], 0.005, 100, 25.0)
    ga = op.table_cell_cross_section(a, F04_T, F04_P, 1990.0, 4001, tab)
    gb = op.table_cell_cross_section(b, F04_T, F04_P, 1990.0, 4001, tab)
    sa, sb = _widths(a)[0], _widths(b)[0]
    np.testing.assert_allclose(gb[1:] / sb, ga[:-1] / sa, rtol=1e-15, atol=0)


def test_table_mode_nearest_node_is_nearest_in_ratio():
    nodes = np.array([1.0, 2.0, 4.0, 8.0])
    x = np.array([0.5, 1.4, 1.42, 2.9, 2.8, 5.6, 5.7, 100.0])
    # midpoints sqrt(2) = 1.414..., sqrt(8) = 2.828..., sqrt(32) = 5.657...
    assert list(op.nearest_node(x, nodes)) == [0, 0, 1, 2, 1, 2, 3, 3]


def test_table_mode_sums_coincident_strengths():
    # item 5: lines sharing profile and shift act as one line with the summed strength
    a = _single_line(nu0=2000.1, s=1e-20)
    two = LineList(np.array([2000.1, 2000.1]), np.array([1e-20, 3e-21]), np.array([0.07, 0.07]),
                   np.array([300.0, 300.0]), np.array([18.015, 18.015]))
    one = _single_line(nu0=2000.1, s=1.3e-20)
    _, sig, gam = _widths(a)
    tab = op.profile_table([sig], [gam], 0.005, 100, 25.0)
    g2 = op.table_cell_cross_section(two, F04_T, F04_P, 1990.0, 4001, tab)
    g1 = op.table_cell_cross_section(one, F04_T, F04_P, 1990.0, 4001, tab)
    np.testing.assert_allclose(g2, g1, rtol=1e-14, atol=0)


def test_table_mode_strength_cutoff():
    # item 6: lines below the threshold relative to the strongest line are ignored
    strong, weak = _single_line(nu0=2000.1, s=1e-20), _single_line(nu0=2003.2, s=1e-23)
    both = LineList(*(np.concatenate([getattr(strong, f), getattr(weak, f)])
                      for f in ("nu0", "s296", "gamma296", "elow", "mass_amu")))
    _, sig, gam = _widths(strong)
    tab = op.profile_table([sig], [gam], 0.005, 100, 25.0)
    args = (F04_T, F04_P, 1990.0, 4001, tab)
    g_s = op.table_cell_cross_section(strong, *args)
    g_w = op.table_cell_cross_section(weak, *args)
    assert np.array_equal(op.table_cell_cross_section(both, *args, strength_cutoff=1e-2), g_s)
    np.testing.assert_allclose(op.table_cell_cross_section(both, *args, strength_cutoff=1e-4), g_s + g_w,
                               rtol=1e-15, atol=0)


def test_table_mode_meets_the_f04_accuracy_bar():
    # Sec. 6.1.1: with a 60 x 60 profile grid the table mode stays within 0.1 % of the
    # directly evaluated profile; here the line's widths are nodes and its centre falls
    # between fine samples (thousands per output interval), so only the shift rounds
    ln = _single_line(nu0=2000.123456)
    _, sig, gam = _widths(ln)
    r = 1.05 ** np.arange(-30, 30)
    tab = op.profile_table(sig * r, gam * r, 0.005, 2000, 25.0)
    assert tab["sigma_nodes"][30] == sig and tab["gamma_nodes"][30] == gam
    got = op.table_cell_cross_section(ln, F04_T, F04_P, 1999.0, 451, tab)
    ref = op.cell_cross_section(ln, F04_T, F04_P, 1999.0, 0.005, 451)
    big = ref > 1e-3 * ref.max()
    assert np.max(np.abs(got[big] - ref[big]) / ref[big]) < 1e-3
