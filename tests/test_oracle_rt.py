"""Pins of the oracle's atmosphere and transmission arithmetic against closed forms,
limits and invariants (Sec. 3, Sec. 6.1, Sec. 6.2)."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import expn

from oracle import atmosphere as atm
from oracle import rt
from oracle.constants import K_B, M_U, BAR
import workloads as wl

PL = wl.Planet()


def _radii_geometric(L, r0=8.0e9, r_top=8.5e9):
    return np.linspace(r0, r_top, L)


# ------------------------------------------------------------------ chord optical depth
def test_uniform_extinction_gives_exact_chord():
    # uniform e: tau_j = 2 e sqrt(R_top^2 - b_j^2), exactly for the trapezoid in s
    L = 37
    r = np.sort(8.0e9 + 4.0e8 * np.random.default_rng(3).random(L))
    e = np.full((L, 3), [1e-9, 3e-7, 2e-5])
    tau = rt.optical_depth(r, e)
    exact = 2 * e[0][None, :] * np.sqrt(r[-1] ** 2 - r[:, None] ** 2)
    np.testing.assert_allclose(tau, exact, rtol=1e-12, atol=0)


def test_tau_monotone_in_impact_parameter():
    # extinction non-increasing outward -> tau non-increasing in b
    L = 40
    r = _radii_geometric(L)
    e = np.exp(-np.arange(L) / 4.0)[:, None] * np.array([[1e-6, 1e-3]])
    tau = rt.optical_depth(r, e)
    assert np.all(np.diff(tau, axis=0) <= 0.0)
    assert np.all(tau[-1] == 0.0)


def test_tau_single_layer_slab():
    # extinction only in one shell [r_m, r_{m+1}]: the ray tangent at r_m crosses the
    # shell over its full chord; trapezoid pieces reduce to s_{m,m+1} (e_m + e_{m+1})
    L, m = 10, 4
    r = _radii_geometric(L)
    e = np.zeros((L, 1))
    e[m] = 2e-7
    tau = rt.optical_depth(r, e)
    s = math.sqrt(r[m + 1] ** 2 - r[m] ** 2)
    assert tau[m, 0] == pytest.approx(s * 2e-7, rel=1e-13)
    assert np.all(tau[m + 1:] == 0.0)


# ------------------------------------------------------------------ transit depth
def test_opaque_disk_depth():
    # no extinction -> depth = (r_0 / Rs)^2 exactly
    L = 25
    r = _radii_geometric(L)
    tau = np.zeros((L, 4))
    d = rt.transit_depth(r, tau, PL.rs_cm)
    np.testing.assert_allclose(d, (r[0] / PL.rs_cm) ** 2, rtol=1e-15)


def test_saturated_depth():
    # tau -> infinity below the top layer -> depth = r_{L-2} r_{L-1} / Rs^2
    L = 25
    r = _radii_geometric(L)
    tau = np.full((L, 2), 1e6)
    tau[-1] = 0.0
    d = rt.transit_depth(r, tau, PL.rs_cm)
    np.testing.assert_allclose(d, r[-2] * r[-1] / PL.rs_cm ** 2, rtol=1e-14)


def test_uniform_extinction_depth_converges_at_order_1p5():
    # closed form for uniform e: Rs^2 depth = R_top^2 - 2 [1 - (1 + kU) e^{-kU}] / k^2,
    # k = 2e, U = sqrt(R_top^2 - r_0^2). tau(b) ~ sqrt(R_top - b) near the top, so the
    # trapezoid in b converges as h^1.5 (error ratio 2^1.5 per halving), not h^2
    r0, rt_ = 8.0e9, 8.05e9
    e = 2e-9
    k, U = 2 * e, math.sqrt(rt_ ** 2 - r0 ** 2)
    exact = (rt_ ** 2 - 2 * (1 - (1 + k * U) * math.exp(-k * U)) / k ** 2) / PL.rs_cm ** 2
    errs = []
    for L in (400, 800, 1600):
        r = np.linspace(r0, rt_, L)
        tau = (2 * e * np.sqrt(rt_ ** 2 - r ** 2))[:, None]   # exact chords (pinned above)
        d = rt.transit_depth(r, tau, PL.rs_cm)[0]
        errs.append(abs(d - exact) / (exact - (r0 / PL.rs_cm) ** 2))
    assert errs[-1] < 2e-5
    assert errs[0] / errs[1] == pytest.approx(2 ** 1.5, rel=0.03)
    assert errs[1] / errs[2] == pytest.approx(2 ** 1.5, rel=0.03)


def test_depth_bounds():
    L = 30
    r = _radii_geometric(L)
    tau = np.abs(np.random.default_rng(1).normal(size=(L, 50))) * 3
    d = rt.transit_depth(r, tau, PL.rs_cm)
    assert np.all(d >= (r[0] / PL.rs_cm) ** 2)
    assert np.all(d <= (r[-1] / PL.rs_cm) ** 2)


def test_thin_limit_linearity():
    # transmission analogue of f05abundance (Sec. 6.1.2, Table 3): for tau << 1 the
    # absorbed part of the depth scales with abundance; the ratio falls slightly below the
    # abundance ratio, by an amount of the order of tau (second-order term of 1 - e^-tau)
    L = 30
    r = _radii_geometric(L)
    shape = np.exp(-np.arange(L) / 5.0)[:, None]
    base = rt.transit_depth(r, np.zeros((L, 1)), PL.rs_cm)[0]
    e1 = 1e-13 * shape
    d1 = rt.transit_depth(r, rt.optical_depth(r, e1), PL.rs_cm)[0] - base
    taumax = rt.optical_depth(r, e1).max()
    for f in range(2, 11):
        df = rt.transit_depth(r, rt.optical_depth(r, f * e1), PL.rs_cm)[0] - base
        ratio = df / d1
        assert ratio < f
        assert f - ratio < f * f * taumax


# ------------------------------------------------------------------ extinction
def test_extinction_interpolation_exact_for_linear_tables():
    S, L, N = 2, 5, 7
    tg = np.array([500.0, 900.0, 1500.0, 2500.0])
    a = np.random.default_rng(2).random((S, 1, L, N)) * 1e-22
    b = np.random.default_rng(3).random((S, 1, L, N)) * 1e-25
    sigma = a + b * tg[None, :, None, None]
    temp = np.array([500.0, 777.0, 1499.0, 2000.0, 2500.0])
    n = np.random.default_rng(4).random((S, L)) * 1e15
    e, flags = rt.extinction(sigma, tg, temp, n)
    expect = np.einsum("sl,sln->ln", n, a[:, 0] + b[:, 0] * temp[None, :, None])
    np.testing.assert_allclose(e, expect, rtol=1e-13)
    assert flags == 0


def test_extinction_clamps_and_flags():
    tg = np.array([500.0, 1000.0])
    sigma = np.array([[[[1.0]], [[3.0]]]])          # [1][2][1][1]
    e, f = rt.extinction(sigma, tg, np.array([200.0]), np.array([[2.0]]))
    assert e[0, 0] == 2.0 and f & atm.FLAG_T_CLAMP
    e, f = rt.extinction(sigma, tg, np.array([4000.0]), np.array([[2.0]]))
    assert e[0, 0] == 6.0 and f & atm.FLAG_T_CLAMP
    e, f = rt.extinction(sigma, tg, np.array([1000.0]), np.array([[2.0]]))
    assert e[0, 0] == 6.0 and f == 0


def test_cia_scales_with_density_squared():
    tg = np.array([500.0, 1000.0])
    sigma = np.zeros((1, 2, 1, 3))
    cia = np.array([[1e-45, 2e-45, 3e-45], [3e-45, 4e-45, 5e-45]])
    e1, _ = rt.extinction(sigma, tg, np.array([750.0]), np.zeros((1, 1)), cia, tg,
                          np.array([1e19]))
    e2, _ = rt.extinction(sigma, tg, np.array([750.0]), np.zeros((1, 1)), cia, tg,
                          np.array([2e19]))
    np.testing.assert_allclose(e2, 4 * e1, rtol=1e-15)
    np.testing.assert_allclose(e1[0], 1e38 * np.array([2e-45, 3e-45, 4e-45]), rtol=1e-14)


def test_binning():
    d = np.arange(95, dtype=float)
    b = rt.bin_spectrum(d, 10)
    assert b.size == 9
    np.testing.assert_allclose(b, np.arange(9) * 10 + 4.5)


# ------------------------------------------------------------------ atmosphere
def test_isothermal_radii_closed_form():
    # T, mu constant: 1/r = 1/R_ref + k_B T / (GM mu m_u) ln(p / p_ref)
    p = wl.layer_pressures(50)
    T = 1234.0
    mu = 2.5
    r, f = atm.radii(p, np.full(p.size, T), mu, 1.1 * wl.R_JUP_CM, PL)
    gm = PL.g_nom * PL.r_nom_cm ** 2
    inv = 1 / (1.1 * wl.R_JUP_CM) + K_B * T / (gm * mu * M_U) * np.log(p / PL.p_ref_bar)
    np.testing.assert_allclose(r, 1 / inv, rtol=1e-14)
    assert f == 0
    assert np.all(np.diff(r) > 0)


def test_radii_linear_profile_exact():
    # T linear in ln p: the trapezoid integral is exact
    p = wl.layer_pressures(31)
    lnp = np.log(p)
    T = 1000.0 + 30.0 * (lnp - math.log(PL.p_ref_bar))
    mu = 2.3
    r, _ = atm.radii(p, T, mu, 1.2 * wl.R_JUP_CM, PL)
    gm = PL.g_nom * PL.r_nom_cm ** 2
    x = lnp - math.log(PL.p_ref_bar)
    integral = 1000.0 * x + 15.0 * x ** 2
    inv = 1 / (1.2 * wl.R_JUP_CM) + K_B / (gm * mu * M_U) * integral
    np.testing.assert_allclose(r, 1 / inv, rtol=1e-13)


def test_expn2_against_its_integral():
    for x in (1e-6, 0.03, 0.7, 3.0, 20.0):
        val, _ = integrate.quad(lambda t: math.exp(-x * t) / t ** 2, 1, np.inf, epsrel=1e-13)
        assert expn(2, x) == pytest.approx(val, rel=1e-11)


def test_line2013_top_of_atmosphere_limit():
    # tau -> 0: xi -> 2/3 + 2 gamma / 3, T^4 -> T_int^4 / 2 + 3/4 T_irr^4 [...]
    tp = np.array([-3.0, -0.5, 0.3, 0.4, 0.9])
    p = np.array([1e-14])
    T = atm.temperature_line2013(p, tp, PL)[0]
    g1, g2, al, be = 10 ** -0.5, 10 ** 0.3, 0.4, 0.9
    tirr = be * math.sqrt(PL.rstar_cm / (2 * PL.a_cm)) * PL.tstar
    t4 = PL.tint ** 4 / 2 + 0.75 * tirr ** 4 * ((1 - al) * (2 / 3 + 2 * g1 / 3)
                                                 + al * (2 / 3 + 2 * g2 / 3))
    assert T == pytest.approx(t4 ** 0.25, rel=1e-9)


def test_line2013_deep_limit():
    # gamma tau >> 1: xi -> 2/3 + 2/(3 gamma); the internal term grows as 3/4 T_int^4 tau
    tp = np.array([0.0, 0.5, 0.8, 0.3, 1.1])
    p = np.array([100.0])
    T = atm.temperature_line2013(p, tp, PL)[0]
    tau = 1.0 * 100.0 * BAR / PL.g_nom
    g1, g2, al, be = 10 ** 0.5, 10 ** 0.8, 0.3, 1.1
    tirr = be * math.sqrt(PL.rstar_cm / (2 * PL.a_cm)) * PL.tstar
    t4 = (0.75 * PL.tint ** 4 * (2 / 3 + tau)
          + 0.75 * tirr ** 4 * ((1 - al) * (2 / 3 + 2 / (3 * g1)) + al * (2 / 3 + 2 / (3 * g2))))
    assert T == pytest.approx(t4 ** 0.25, rel=1e-12)


def test_irradiation_temperature_matches_hot_jupiter():
    # beta = 1 for the HD 189733 b-like system gives T_irr ~ 1190 K (the "~1100 K"
    # mean temperatures of the comparison tests, Table 1)
    tirr = math.sqrt(PL.rstar_cm / (2 * PL.a_cm)) * PL.tstar
    assert 1150 < tirr < 1220


def test_composition_filler():
    x, xh2, xhe, mu, f = atm.composition(np.array([-30.0]), np.array([18.0]), PL)
    assert mu == pytest.approx(0.85 * 2.01588 + 0.15 * 4.002602, rel=1e-12)
    assert f == 0
    x, xh2, xhe, mu, f = atm.composition(np.array([-0.1, -0.2]), np.array([18.0, 44.0]), PL)
    assert f & atm.FLAG_SUM_X and xh2 == 0.0 and xhe == 0.0


def test_forward_isothermal_monotone_and_bounded():
    s = wl.config1()
    s.nu = s.nu[:40]
    sigma = wl.random_opacity_table(1, s.temps, s.p_bar.size, s.nu, seed=5)
    out = rt.forward(wl.config1_params(), s, sigma)
    r = out["atm"]["radius"]
    assert out["flags"] == 0
    assert np.all(np.diff(out["tau"], axis=0) <= 0)
    assert np.all(out["depth"] >= (r[0] / s.planet.rs_cm) ** 2)
    assert np.all(out["depth"] <= (r[-1] / s.planet.rs_cm) ** 2)


def test_optical_depth_limit_saturates_the_chords_below():
    # a limit below every nonzero optical depth makes every chord but the top one opaque:
    # the same closed form as an infinitely opaque atmosphere
    L = 25
    r = _radii_geometric(L)
    g = np.random.default_rng(7)
    tau = np.sort(g.uniform(1e-3, 3.0, (L, 3)), axis=0)[::-1].copy()
    tau[-1] = 0.0
    d = rt.transit_depth(r, tau, PL.rs_cm, tau_max=1e-6)
    np.testing.assert_allclose(d, r[-2] * r[-1] / PL.rs_cm ** 2, rtol=1e-14)


def test_optical_depth_limit_effect_and_limits():
    L = 30
    r = _radii_geometric(L)
    e = np.full((L, 4), 2e-10)
    tau = rt.optical_depth(r, e)
    base = rt.transit_depth(r, tau, PL.rs_cm)
    # an unreachable limit changes nothing
    np.testing.assert_array_equal(rt.transit_depth(r, tau, PL.rs_cm, tau_max=1e30), base)
    # the limit only makes chords more opaque; its effect on a chord is at most exp(-tau_max)
    for tm in (0.5, 2.0, 5.0):
        d = rt.transit_depth(r, tau, PL.rs_cm, tau_max=tm)
        assert np.all(d >= base)
        area = (r[-1] ** 2 - r[0] ** 2) / PL.rs_cm ** 2
        assert np.all(d - base <= np.exp(-tm) * area + 1e-18)
    # with the optical depth monotone in impact parameter, the top-down rule equals the
    # per-chord threshold f = 1 where tau >= tau_max
    tm = 1.0
    f = np.where(tau >= tm, 1.0, -np.expm1(-tau))
    acc = np.full(4, r[0] ** 2)
    for j in range(L - 1):
        acc += (r[j + 1] - r[j]) * (f[j] * r[j] + f[j + 1] * r[j + 1])
    np.testing.assert_allclose(rt.transit_depth(r, tau, PL.rs_cm, tau_max=tm), acc / PL.rs_cm ** 2,
                               rtol=1e-15)


def test_optical_depth_limit_scans_from_the_top():
    # a non-monotone optical depth (not produced by the model, built by hand): a chord
    # above the first one to reach the limit keeps its own absorption; every chord below
    # it is opaque even where its own tau is small
    r = _radii_geometric(5)
    tau = np.array([[0.1], [0.2], [5.0], [0.3], [0.0]])
    d = rt.transit_depth(r, tau, PL.rs_cm, tau_max=1.0)
    f = np.array([1.0, 1.0, 1.0, -np.expm1(-0.3), 0.0])
    acc = r[0] ** 2 + sum((r[j + 1] - r[j]) * (f[j] * r[j] + f[j + 1] * r[j + 1]) for j in range(4))
    assert d[0] == pytest.approx(acc / PL.rs_cm ** 2, rel=1e-15)


def test_rayleigh_h2_cross_section():
    # the inverse-fourth-power law at long wavelengths, positive and falling with
    # wavelength, and the wavelength corrections small in the visible
    nu = np.array([10.0, 20.0])          # 1e7 and 5e6 Angstrom
    s = rt.rayleigh_h2(nu)
    assert s[1] / s[0] == pytest.approx(16.0, rel=1e-6)
    nus = np.linspace(1000.0, 25000.0, 50)
    sr = rt.rayleigh_h2(nus)
    assert np.all(sr > 0) and np.all(np.diff(sr) > 0)
    lam = 1e8 / 20000.0                  # 5000 Angstrom
    leading = 8.14e-13 / lam ** 4
    assert 1.0 < rt.rayleigh_h2(np.array([20000.0]))[0] / leading < 1.1


def test_rayleigh_h2_leading_coefficient_from_refractivity():
    # the Rayleigh cross section of a gas from its refractive index (Lorenz-Lorentz):
    # sigma = 24 pi^3 / (lam^4 N^2) ((n^2 - 1) / (n^2 + 2))^2 at the number density N of the
    # refractivity measurement (0 C, 1 atm: Loschmidt N = 2.6868e19 cm^-3). Published H2
    # refractivities there are n - 1 = 1.32e-4 to 1.36e-4 at long wavelengths and up to
    # 1.40e-4 at 5000 A; the depolarisation (King) correction adds a few per cent. The
    # expansion must fall inside that band, widened by -5 % / +10 %; a wrong power of ten,
    # a wrong wavelength unit or a dropped pi^3 falls far outside it.
    N = 2.6868e19

    def lorenz(n_minus_1, lam_cm):
        n2 = (1.0 + n_minus_1) ** 2
        return 24 * math.pi ** 3 / (lam_cm ** 4 * N ** 2) * ((n2 - 1) / (n2 + 2)) ** 2

    lam_a = 1.0e7                        # 1 mm: the lam^-6 and lam^-8 terms are negligible
    got = rt.rayleigh_h2(np.array([1e8 / lam_a]))[0]
    assert 0.95 * lorenz(1.32e-4, lam_a * 1e-8) <= got <= 1.10 * lorenz(1.36e-4, lam_a * 1e-8)
    got5 = rt.rayleigh_h2(np.array([20000.0]))[0]   # 5000 A, the whole expansion
    assert 0.95 * lorenz(1.36e-4, 5000e-8) <= got5 <= 1.10 * lorenz(1.40e-4, 5000e-8)


def test_cloud_layer_index():
    p = np.logspace(2, -8, 11)            # 100 ... 1e-8 bar, deepest first
    assert rt.cloud_layer(p, 3.0) == -1   # below every layer
    assert rt.cloud_layer(p, 2.0) == 0
    assert rt.cloud_layer(p, -2.0) == 4   # p_4 = 1e-2 bar
    assert rt.cloud_layer(p, -2.5) == 4
    assert rt.cloud_layer(p, -9.0) == 10


def test_cloud_deck_limits_and_monotonicity():
    L = 20
    r = _radii_geometric(L)
    g = np.random.default_rng(11)
    tau = np.sort(g.uniform(0.0, 2.0, (L, 3)), axis=0)[::-1].copy()
    tau[-1] = 0.0
    clear = rt.transit_depth(r, tau, PL.rs_cm)
    # a deck below the deepest layer changes nothing; a deck at the top is a saturated disk
    np.testing.assert_array_equal(rt.transit_depth(r, tau, PL.rs_cm, cloud_index=-1), clear)
    np.testing.assert_allclose(rt.transit_depth(r, tau, PL.rs_cm, cloud_index=L - 1),
                               r[-1] ** 2 / PL.rs_cm ** 2, rtol=1e-14)
    # a higher cloud top only adds absorption
    prev = clear
    for jc in range(L):
        d = rt.transit_depth(r, tau, PL.rs_cm, cloud_index=jc)
        assert np.all(d >= prev - 1e-18)
        prev = d


def _helium_case(h2_frac, seed=3):
    """A small isothermal atmosphere with the given H2 share of the filler gas."""
    import dataclasses
    pl = dataclasses.replace(wl.Planet(), h2_frac=h2_frac)
    p_bar = wl.layer_pressures(12)
    mass = wl.ABSORBER_MASS_AMU[:2].copy()
    a = atm.atmosphere(np.array([1300.0, -3.0, -4.0, 1.1]), p_bar, mass, 0, pl)
    temps = np.linspace(500.0, 3000.0, 6)
    nu = np.linspace(1000.0, 9000.0, 40)
    g = np.random.default_rng(seed)
    sigma = g.uniform(1e-24, 1e-22, size=(2, temps.size, p_bar.size, nu.size))
    return a, temps, nu, sigma


def test_h2he_cia_vanishes_without_helium():
    # an all-H2 filler has n_He = 0: the H2-He term adds nothing
    a, temps, nu, sigma = _helium_case(1.0)
    k1, k2 = wl.cia_table(temps, nu), wl.cia_he_table(temps, nu)
    e0, _ = rt.extinction(sigma, temps, a["temp"], a["n_species"], k1, temps, a["n_h2"])
    e1, _ = rt.extinction(sigma, temps, a["temp"], a["n_species"], k1, temps, a["n_h2"], k2, a["n_he"])
    assert np.all(a["n_he"] == 0.0) and np.array_equal(e0, e1)


def test_h2he_cia_at_equal_filler_shares_is_the_h2h2_form():
    # with H2:He = 1:1 the densities agree, n_H2 n_He = n_H2^2, so the H2-He term with
    # table K equals the (separately pinned) H2-H2 term with the same table
    a, temps, nu, sigma = _helium_case(0.5)
    np.testing.assert_allclose(a["n_he"], a["n_h2"], rtol=1e-15)
    k2 = wl.cia_he_table(temps, nu)
    zero = np.zeros_like(k2)
    e_he, _ = rt.extinction(sigma, temps, a["temp"], a["n_species"], zero, temps, a["n_h2"], k2, a["n_he"])
    e_hh, _ = rt.extinction(sigma, temps, a["temp"], a["n_species"], k2, temps, a["n_h2"])
    np.testing.assert_allclose(e_he, e_hh, rtol=1e-14)


def test_cia_tables_combine_into_one_h2h2_table():
    # n_He / n_H2 = (1 - h) / h in every layer, so both CIA terms equal one H2-H2 term
    # with the table K_H2H2 + ((1 - h) / h) K_H2He
    h = 0.85
    a, temps, nu, sigma = _helium_case(h)
    np.testing.assert_allclose(a["n_he"] / a["n_h2"], (1 - h) / h, rtol=1e-14)
    k1, k2 = wl.cia_table(temps, nu), wl.cia_he_table(temps, nu)
    e_sep, _ = rt.extinction(sigma, temps, a["temp"], a["n_species"], k1, temps, a["n_h2"], k2, a["n_he"])
    e_one, _ = rt.extinction(sigma, temps, a["temp"], a["n_species"], k1 + (1 - h) / h * k2, temps, a["n_h2"])
    np.testing.assert_allclose(e_sep, e_one, rtol=1e-13)
    # and the H2-He term is not negligible in the band it covers
    e_hh, _ = rt.extinction(sigma, temps, a["temp"], a["n_species"], k1, temps, a["n_h2"])
    assert np.max((e_sep - e_hh) / e_hh) > 1e-3


# ---- emission (eclipse) geometry ---------------------------------------------------------
def test_planck_wien_peak_and_stefan_boltzmann():
    # the peak of B_nu (per wavenumber) sits at x = c2 nu / T solving 3 (1 - e^-x) = x
    # (Wien's law for this form, Sec. 6 f08 test); its integral is sigma T^4 / pi
    from scipy import optimize
    x_w = optimize.brentq(lambda x: 3.0 * (1.0 - math.exp(-x)) - x, 1.0, 5.0)
    for T in (700.0, 1500.0, 2900.0):
        nu = np.linspace(1.0, 40.0 * T, 400001)
        b = rt.planck(nu, T)
        nu_peak = nu[np.argmax(b)]
        assert nu_peak == pytest.approx(x_w * T / 1.4387769, rel=2e-4)
        total, _ = integrate.quad(lambda v: rt.planck(np.array([v]), T)[0], 1e-6, 60.0 * T, limit=400)
        assert total == pytest.approx(5.670374419e-5 * T ** 4 / math.pi, rel=1e-7)


def _emission_layers(L=40):
    r = np.linspace(8.0e9, 8.3e9, L)
    return r


def test_vertical_optical_depth_exact_for_uniform_extinction():
    r = _emission_layers()
    e = np.full((r.size, 3), 2.5e-9)
    tau = rt.vertical_optical_depth(r, e)
    np.testing.assert_allclose(tau, 2.5e-9 * (r[-1] - r)[:, None] * np.ones(3), rtol=1e-13, atol=1e-18)


def test_isothermal_atmosphere_emits_a_blackbody():
    # f08isothermal (Sec. 6): an isothermal atmosphere of any opacity emits B(T) exactly
    r = _emission_layers()
    nu = np.linspace(500.0, 9000.0, 50)
    g = np.random.default_rng(2)
    ext = g.uniform(0.0, 3e-8, size=(r.size, nu.size))
    tau = rt.vertical_optical_depth(r, ext)
    got = rt.emergent_intensity(np.full(r.size, 1234.5), tau, nu)
    np.testing.assert_allclose(got, rt.planck(nu, 1234.5), rtol=1e-13)


def test_transparent_atmosphere_shows_the_deep_blackbody_and_two_layer_closed_form():
    nu = np.linspace(500.0, 9000.0, 20)
    r = np.array([8.0e9, 8.0e9 + 3.0e6])
    temp = np.array([1600.0, 900.0])
    tau0 = rt.vertical_optical_depth(r, np.zeros((2, nu.size)))
    np.testing.assert_array_equal(rt.emergent_intensity(temp, tau0, nu), rt.planck(nu, 1600.0))
    e = np.full((2, nu.size), 4e-7)
    t = 4e-7 * 3.0e6
    b0, b1 = rt.planck(nu, 1600.0), rt.planck(nu, 900.0)
    want = b0 * math.exp(-t) + 0.5 * (b0 + b1) * (1.0 - math.exp(-t))
    np.testing.assert_allclose(rt.emergent_intensity(temp, rt.vertical_optical_depth(r, e), nu), want,
                               rtol=1e-14)


def test_emission_thin_limit_linearity():
    # f05abundance (Sec. 6, Table 3): in the optically thin limit the absorbed fraction
    # scales with the absorber abundance, f = (F0 - Fh) / (F0 - Fl) -> x_h / x_l; with
    # saturation the ratio falls slightly below f, more so for larger f (as in Table 3)
    L = 40
    r = _emission_layers(L)
    temp = np.linspace(1500.0, 900.0, L)       # non-inverted: cooler upward
    nu = np.linspace(1990.0, 2010.0, 201)
    line = 1e-7 * np.exp(-((nu - 2000.0) / 0.5) ** 2)   # extinction per unit abundance, cm^-1
    base = np.full(L, 1e-10)[:, None] * np.ones(nu.size)
    def spectrum(x):
        ext = base + x * np.ones(L)[:, None] * line[None, :]
        return rt.emergent_intensity(temp, rt.vertical_optical_depth(r, ext), nu)
    f0, fl = spectrum(0.0), spectrum(1e-5)
    c = np.argmin(np.abs(nu - 2000.0))
    ratios = []
    for f in range(2, 11):
        fh = spectrum(f * 1e-5)
        ratios.append((f0[c] - fh[c]) / (f0[c] - fl[c]))
    ratios = np.array(ratios)
    fs = np.arange(2, 11)
    assert np.all(ratios < fs) and np.all(np.abs(ratios - fs) / fs < 2e-3)
    assert np.all(np.diff(fs - ratios) > 0)
