"""Atmosphere model of the forward model (oracle; test infrastructure only).

Steps a1-a2 of the hot path: the profile generator turns a parameter vector into
a temperature, composition and number density per layer (Sec. 3, Fig. 1), and the
layers are placed at radii by hydrostatic balance anchored at the reference
pressure where the radius parameter applies (Sec. 6.2: radius given at 0.1 bar).

Parameter vector
  tp_mode 0 (isothermal):  [T, log10 x_1..x_S, R_ref/R_J]
  tp_mode 1 (Line 2013):   [log10 kappa, log10 gamma1, log10 gamma2, alpha, beta,
                            log10 x_1..x_S, R_ref/R_J]
(Sec. 6.3 and Sec. 7: five T(p) parameters of Line et al. 2013, all base-10
logarithms except alpha and beta; constant-with-height log abundances; a radius
at the reference pressure for transmission.)
"""
from __future__ import annotations

import math
import numpy as np
from scipy.special import expn

from .constants import K_B, M_U, G_GRAV, BAR

R_JUP_CM = 7.1492e9

FLAG_T_CLAMP = 1        # a layer temperature fell outside a table's temperature range
FLAG_SUM_X = 2          # the absorber mixing ratios sum to 1 or more
FLAG_RADIUS = 4         # hydrostatic radius became invalid (1/r <= 0)
FLAG_NONFINITE = 8      # non-finite parameter or temperature


def n_tp_params(tp_mode: int) -> int:
    return 1 if tp_mode == 0 else 5


def xi_line2013(gamma: float, tau: np.ndarray) -> np.ndarray:
    """Irradiation-stream function of the Line et al. (2013) / Guillot (2010) profile:
    xi = 2/3 + 2/(3 gamma) [1 + (gamma tau / 2 - 1) exp(-gamma tau)]
             + (2 gamma / 3) (1 - tau^2 / 2) E2(gamma tau)."""
    gt = gamma * tau
    return (2.0 / 3.0
            + 2.0 / (3.0 * gamma) * (1.0 + (gt / 2.0 - 1.0) * np.exp(-gt))
            + 2.0 * gamma / 3.0 * (1.0 - tau ** 2 / 2.0) * expn(2, gt))


def temperature_line2013(p_bar: np.ndarray, tp: np.ndarray, planet) -> np.ndarray:
    """Five-parameter T(p) of Line et al. (2013), as used by BART (Sec. 6.3, Sec. 7).

    tau = kappa p / g;  T_irr = beta sqrt(R_star / (2 a)) T_star;
    T^4 = 3/4 T_int^4 (2/3 + tau) + 3/4 T_irr^4 (1 - alpha) xi(gamma1)
          + 3/4 T_irr^4 alpha xi(gamma2).
    """
    kappa = 10.0 ** tp[0]
    g1 = 10.0 ** tp[1]
    g2 = 10.0 ** tp[2]
    alpha = tp[3]
    beta = tp[4]
    tau = kappa * (p_bar * BAR) / planet.g_nom
    t_irr = beta * math.sqrt(planet.rstar_cm / (2.0 * planet.a_cm)) * planet.tstar
    t4 = (0.75 * planet.tint ** 4 * (2.0 / 3.0 + tau)
          + 0.75 * t_irr ** 4 * (1.0 - alpha) * xi_line2013(g1, tau)
          + 0.75 * t_irr ** 4 * alpha * xi_line2013(g2, tau))
    return t4 ** 0.25


def composition(log_x: np.ndarray, mass_amu: np.ndarray, planet):
    """Absorber mixing ratios x_i = 10^theta_i, the H2/He filler taking the remainder
    in the ratio 0.85:0.15, and the mean molecular mass in amu.
    Returns (x[S], x_h2, x_he, mu, flags)."""
    x = 10.0 ** np.asarray(log_x, dtype=np.float64)
    total = float(np.sum(x))
    flags = FLAG_SUM_X if total >= 1.0 else 0
    fill = max(0.0, 1.0 - total)
    x_h2 = planet.h2_frac * fill
    x_he = (1.0 - planet.h2_frac) * fill
    mu = float(np.sum(x * mass_amu)) + x_h2 * planet.m_h2_amu + x_he * planet.m_he_amu
    return x, x_h2, x_he, mu, flags


def number_density(p_bar: np.ndarray, temp: np.ndarray) -> np.ndarray:
    """Ideal gas: n = p / (k_B T), molecules cm^-3."""
    return p_bar * BAR / (K_B * temp)


def _interp_lnp(lnp_desc: np.ndarray, values: np.ndarray, target: float) -> float:
    """Linear interpolation in ln p on a grid ordered deepest (largest p) first."""
    return float(np.interp(target, lnp_desc[::-1], values[::-1]))


def radii(p_bar: np.ndarray, temp: np.ndarray, mu: float, r_ref_cm: float, planet):
    """Hydrostatic layer radii with g = GM / r^2, GM = g_nom r_nom^2.

    dp/p = -(mu m_u GM / (k_B T)) dr / r^2  gives
    1/r(p) = 1/R_ref + k_B / (GM mu m_u) * integral_{ln p_ref}^{ln p} T d ln p',
    the integral taken exactly for the piecewise-linear (in ln p) temperature profile
    through the layer nodes; T at p_ref is interpolated linearly in ln p.
    Returns (r[L] in cm, flags)."""
    lnp = np.log(p_bar)
    ln_ref = math.log(planet.p_ref_bar)
    if not (lnp.min() <= ln_ref <= lnp.max()):
        raise ValueError("reference pressure outside the layer grid")
    gm = planet.g_nom * planet.r_nom_cm ** 2
    coef = K_B / (gm * mu * M_U)
    r = np.empty_like(p_bar)
    flags = 0
    for l in range(p_bar.size):
        a, b = ln_ref, lnp[l]
        lo, hi = min(a, b), max(a, b)
        inner = sorted(v for v in lnp if lo < v < hi)
        pts = [a] + (inner if b > a else inner[::-1]) + [b]
        tpts = [_interp_lnp(lnp, temp, v) for v in pts]
        integral = 0.0
        for i in range(len(pts) - 1):
            integral += (pts[i + 1] - pts[i]) * 0.5 * (tpts[i] + tpts[i + 1])
        inv_r = 1.0 / r_ref_cm + coef * integral
        if not inv_r > 0.0:
            flags |= FLAG_RADIUS
            r[l] = math.nan
        else:
            r[l] = 1.0 / inv_r
    return r, flags


def atmosphere(params: np.ndarray, p_bar: np.ndarray, mass_amu: np.ndarray, tp_mode: int, planet):
    """Steps a1-a2: parameter vector -> per-layer T, absorber number densities,
    H2 number density, radii and status flags (all float64)."""
    params = np.asarray(params, dtype=np.float64)
    S = mass_amu.size
    ntp = n_tp_params(tp_mode)
    flags = 0
    if not np.all(np.isfinite(params)):
        flags |= FLAG_NONFINITE
    if tp_mode == 0:
        temp = np.full(p_bar.size, params[0])
    else:
        temp = temperature_line2013(p_bar, params[:5], planet)
    if not (np.all(np.isfinite(temp)) and np.all(temp > 0.0)):
        flags |= FLAG_NONFINITE
    x, x_h2, x_he, mu, f = composition(params[ntp:ntp + S], mass_amu, planet)
    flags |= f
    n = number_density(p_bar, temp)
    n_species = x[:, None] * n[None, :]
    n_h2 = x_h2 * n
    n_he = x_he * n
    r, f = radii(p_bar, temp, mu, params[ntp + S] * R_JUP_CM, planet)
    flags |= f
    return dict(temp=temp, n_species=n_species, n_h2=n_h2, n_he=n_he, radius=r, mu=mu, x=x,
                x_h2=x_h2, flags=flags)
