"""Seeded synthetic inputs for the transmission forward model and its tests.

This module only *draws inputs*: line lists, grids, opacity and CIA tables,
planet constants and parameter vectors. It holds none of the radiative-transfer
arithmetic; both the GPU library and the CPU oracle consume what it returns.

The paper's workloads use HITRAN/HITEMP/ExoMol line lists, HITRAN CIA tables
and HD 189733 b data (Sec. 7), none of which are available here; the recipes
below stand in for them with the same shapes and value ranges: 100 layers
log-spaced over 1e-8--100 bar (Sec. 7), a hot-Jupiter planet/star pair
(Sec. 6.2), and constant-with-height log abundances (Sec. 6.3, Sec. 7).

Every generator takes an explicit seed and uses numpy's PCG64.
"""
from __future__ import annotations

import dataclasses
import numpy as np

R_JUP_CM = 7.1492e9          # IAU equatorial Jupiter radius (the paper insists on IAU values)
R_SUN_CM = 6.957e10          # IAU nominal solar radius
AU_CM = 1.495978707e13
SEED_BASE = 2104_12522

#: absorber masses in amu, in the order H2O, CO, CO2, CH4 (the HD 189733 b species, Sec. 7)
ABSORBER_MASS_AMU = np.array([18.015, 28.010, 44.009, 16.043])
ABSORBER_NAMES = ("H2O", "CO", "CO2", "CH4")


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------------------
# grids
# --------------------------------------------------------------------------------------
def layer_pressures(n_layers: int, p_bottom_bar: float = 100.0, p_top_bar: float = 1e-8) -> np.ndarray:
    """Layer pressures in bar, log-spaced, index 0 deepest (p_bottom) ... L-1 top."""
    return np.logspace(np.log10(p_bottom_bar), np.log10(p_top_bar), n_layers)


def temperature_grid(n_temp: int, t_min: float, t_max: float) -> np.ndarray:
    return np.linspace(t_min, t_max, n_temp)


def wavenumber_grid(nu_start: float, dnu: float, n_nu: int) -> np.ndarray:
    return nu_start + dnu * np.arange(n_nu, dtype=np.float64)


# --------------------------------------------------------------------------------------
# line lists (structure-of-arrays)
# --------------------------------------------------------------------------------------
@dataclasses.dataclass
class LineList:
    nu0: np.ndarray        # line centre, cm^-1
    s296: np.ndarray       # line strength at 296 K, cm^-1 / (molecule cm^-2)
    gamma296: np.ndarray   # Lorentz HWHM at 1 atm and 296 K, cm^-1
    elow: np.ndarray       # lower-state energy, cm^-1
    mass_amu: np.ndarray   # molecular mass per line, amu

    def __len__(self) -> int:
        return int(self.nu0.size)

    def subset(self, idx) -> "LineList":
        return LineList(*(np.ascontiguousarray(a[idx]) for a in
                          (self.nu0, self.s296, self.gamma296, self.elow, self.mass_amu)))


def line_list(n_lines: int, seed: int, nu_min: float = 1000.0, nu_max: float = 5000.0,
              mass_amu: float | None = 18.015, mass_range=(18.0, 44.0)) -> LineList:
    """Synthetic line list sorted by centre: centres U[nu_min, nu_max], log10 S U[-25,-19],
    Lorentz HWHM U[0.05, 0.1] cm^-1, E'' U[0, 5000] cm^-1. ``mass_amu=None``
    draws a per-line mass U[mass_range] (the opacity-build stress case)."""
    g = rng(seed)
    nu0 = g.uniform(nu_min, nu_max, n_lines)
    s296 = 10.0 ** g.uniform(-25.0, -19.0, n_lines)
    gam = g.uniform(0.05, 0.1, n_lines)
    elow = g.uniform(0.0, 5000.0, n_lines)
    if mass_amu is None:
        mass = g.uniform(mass_range[0], mass_range[1], n_lines)
    else:
        mass = np.full(n_lines, float(mass_amu))
    order = np.argsort(nu0, kind="stable")   # line lists are distributed sorted by centre
    return LineList(nu0[order], s296[order], gam[order], elow[order], mass[order])


# --------------------------------------------------------------------------------------
# tables
# --------------------------------------------------------------------------------------
def cia_table(temps: np.ndarray, nu: np.ndarray) -> np.ndarray:
    """Smooth synthetic H2-H2 CIA coefficient [NTc][Nnu] in cm^5 molecule^-2:
    two Gaussian bands (near the H2 fundamental and first overtone) scaled as T^0.5,
    plus a floor. A stand-in for the HITRAN CIA tables."""
    t = np.asarray(temps, dtype=np.float64)[:, None]
    v = np.asarray(nu, dtype=np.float64)[None, :]
    band = np.exp(-((v - 4160.0) / 600.0) ** 2) + 0.3 * np.exp(-((v - 8300.0) / 900.0) ** 2)
    return 1e-45 * np.sqrt(t / 1000.0) * band + 1e-48


def cia_he_table(temps: np.ndarray, nu: np.ndarray) -> np.ndarray:
    """Smooth synthetic H2-He CIA coefficient [NTc][Nnu] in cm^5 molecule^-2: one broad
    band below the H2 fundamental, growing as T^0.7, plus a floor. A stand-in for the
    HITRAN H2-He table."""
    t = np.asarray(temps, dtype=np.float64)[:, None]
    v = np.asarray(nu, dtype=np.float64)[None, :]
    band = np.exp(-((v - 3800.0) / 900.0) ** 2)
    return 4e-46 * (t / 1000.0) ** 0.7 * band + 5e-49


def random_opacity_table(n_species: int, temps: np.ndarray, n_layers: int, nu: np.ndarray,
                         seed: int, line_density: float = 0.02, dtype=np.float64) -> np.ndarray:
    """Cross-section table [S][NT][L][Nnu] (cm^2/molecule) with line-like spikes on a
    continuum, smooth in T and in pressure. Used where the forward model needs a table
    that neither the GPU nor the oracle produced (forward-model parity at full size)."""
    g = rng(seed)
    nT, nnu = len(temps), len(nu)
    out = np.empty((n_species, nT, n_layers, nnu), dtype=dtype)
    tnorm = ((np.asarray(temps, dtype=np.float64) - temps[0])
             / max(temps[-1] - temps[0], 1.0)).astype(dtype)
    lay = np.linspace(0.0, 1.0, n_layers, dtype=dtype)
    for s in range(n_species):
        base = (10.0 ** g.uniform(-27.0, -24.0, nnu)).astype(dtype)       # continuum, per nu
        spikes = ((g.random(nnu) < line_density)
                  * 10.0 ** g.uniform(-22.0, -19.0, nnu)).astype(dtype)
        tdep = (0.5 + g.random(nnu)).astype(dtype)                         # per-nu T slope
        pdep = (0.3 + 0.7 * g.random(nnu)).astype(dtype)                   # per-nu p smoothing
        prof = base[None, :] + spikes[None, :] * (1 - 0.5 * pdep[None, :] * lay[:, None])
        for it in range(nT):
            out[s, it] = prof * (1 + tdep * tnorm[it])[None, :]
    return out


# --------------------------------------------------------------------------------------
# planet / star / model constants
# --------------------------------------------------------------------------------------
@dataclasses.dataclass
class Planet:
    """Fixed constants of a transmission model (hot Jupiter resembling HD 189733 b,
    Sec. 6.2 and Sec. 7). Lengths in cm, temperatures in K, gravity in cm s^-2."""
    rs_cm: float = 0.756 * R_SUN_CM          # stellar radius
    tstar: float = 5000.0                     # stellar temperature
    rstar_cm: float = 0.756 * R_SUN_CM        # star radius used by the T(p) irradiation term
    a_cm: float = 0.0312 * AU_CM              # semi-major axis
    tint: float = 100.0                       # internal temperature of the T(p) profile
    g_nom: float = 2100.0                     # gravity at the nominal radius
    r_nom_cm: float = 1.14 * R_JUP_CM         # nominal radius fixing GM = g_nom r_nom^2
    p_ref_bar: float = 0.1                    # pressure at which the radius parameter applies
    h2_frac: float = 0.85                     # filler-gas split H2:He
    m_h2_amu: float = 2.01588
    m_he_amu: float = 4.002602


@dataclasses.dataclass
class Prior:
    """Uniform prior box per parameter (log parameters are log-uniform)."""
    lo: np.ndarray
    hi: np.ndarray

    def draw(self, n: int, seed: int) -> np.ndarray:
        g = rng(seed)
        return self.lo + (self.hi - self.lo) * g.random((n, self.lo.size))


def line2013_prior(n_species: int, alpha_max: float = 1.0) -> Prior:
    """Parameters: log10 kappa, log10 gamma1, log10 gamma2, alpha, beta,
    log10 x_i (n_species), R_ref / R_J.

    The profile is unchanged by exchanging the two visible streams, (gamma1, gamma2, alpha)
    -> (gamma2, gamma1, 1 - alpha), and gamma1 and gamma2 share one range, so with
    alpha in [0, 1] every posterior has a mirror mode. alpha_max = 0.5 labels the streams
    (the one with weight 1 - alpha >= alpha is stream 1) and keeps every profile."""
    lo = np.array([-3.0, -1.5, -1.5, 0.0, 0.6] + [-8.0] * n_species + [1.0])
    hi = np.array([0.0, 1.0, 1.0, alpha_max, 1.2] + [-2.0] * n_species + [1.3])
    return Prior(lo, hi)


def with_cloud(prior: Prior, log_p_lo: float = -6.0, log_p_hi: float = 2.0) -> Prior:
    """The prior extended by the cloud-top pressure, log10 p_cloud (bar), last."""
    return Prior(np.append(prior.lo, log_p_lo), np.append(prior.hi, log_p_hi))


def isothermal_prior(n_species: int) -> Prior:
    """Parameters: T (K), log10 x_i (n_species), R_ref / R_J."""
    lo = np.array([800.0] + [-8.0] * n_species + [1.0])
    hi = np.array([2000.0] + [-2.0] * n_species + [1.3])
    return Prior(lo, hi)


# --------------------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------------------
@dataclasses.dataclass
class ForwardSetup:
    name: str
    n_species: int
    temps: np.ndarray
    p_bar: np.ndarray
    nu: np.ndarray
    mass_amu: np.ndarray
    tp_mode: int                 # 0 isothermal, 1 Line et al. (2013) five-parameter profile
    planet: Planet
    cia_temps: np.ndarray | None = None
    bin_width: int = 0
    lines_per_species: tuple = ()
    tau_max: float = 0.0         # optical-depth limit (0: none)
    rayleigh: bool = False       # H2 Rayleigh scattering in the extinction
    cloud: bool = False          # gray cloud deck: one more parameter, log10 p_cloud (bar)
    geometry: str = "transit"    # "transit" (transit depth) or "eclipse" (emergent intensity)


def config1() -> ForwardSetup:
    """FP64 plain forward model: one absorber (1e4 lines), 10 T x 50 p x 1000 nu (4 cm^-1),
    isothermal 1200 K, x = 1e-4, no CIA."""
    return ForwardSetup(
        name="fp64_1abs_50lyr_1k", n_species=1,
        temps=temperature_grid(10, 500.0, 3000.0), p_bar=layer_pressures(50),
        nu=wavenumber_grid(1000.0, 4.0, 1000), mass_amu=ABSORBER_MASS_AMU[:1].copy(),
        tp_mode=0, planet=Planet(), lines_per_species=(10_000,))


def config1_params() -> np.ndarray:
    return np.array([1200.0, -4.0, 1.14])


def config2(n_nu: int = 30000, n_layers: int = 100, dnu: float = 0.5) -> ForwardSetup:
    """Full forward model: 4 absorbers, 20 T (300-3000 K) x 100 p x 30000 nu (0.5 cm^-1
    from 1000 cm^-1), H2-H2 CIA on the same 20 T, five-parameter T(p), 30-point bins."""
    temps = temperature_grid(20, 300.0, 3000.0)
    return ForwardSetup(
        name="fp32_4abs_100lyr_30k", n_species=4, temps=temps,
        p_bar=layer_pressures(n_layers), nu=wavenumber_grid(1000.0, dnu, n_nu),
        mass_amu=ABSORBER_MASS_AMU.copy(), tp_mode=1, planet=Planet(),
        cia_temps=temps.copy(), bin_width=30,
        lines_per_species=(100_000, 250_000, 500_000, 1_000_000))


def config3_mixed():
    """The mixed batch: (L, Nnu, dnu) = (60, 8000, 0.5), (100, 30000, 0.5), (150, 50000, 0.3)."""
    out = []
    for L, n, d in ((60, 8000, 0.5), (100, 30000, 0.5), (150, 50000, 0.3)):
        s = config2(n_nu=n, n_layers=L, dnu=d)
        s.name = f"fp32_4abs_{L}lyr_{n // 1000}k"
        out.append(s)
    return out


def config4_lines(n_lines: int = 10_000_000, seed: int = SEED_BASE + 4) -> LineList:
    """Opacity build stress case: config-1 distributions with per-line mass U[18,44] amu."""
    return line_list(n_lines, seed, mass_amu=None)


def config4_grid():
    """1e5 nu (0.04 cm^-1 from 1000) x 20 T (300-3000) x 100 p (1e-8--100 bar)."""
    return (wavenumber_grid(1000.0, 0.04, 100_000), temperature_grid(20, 300.0, 3000.0),
            layer_pressures(100))
