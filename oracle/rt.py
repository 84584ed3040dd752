"""Transmission radiative transfer of the forward model (oracle; test infrastructure only).

Steps a3-a6 of the hot path (Sec. 3: transit interpolates the pre-computed opacity
table to each layer's temperature, the table lives on the layer pressures and the
output wavenumber grid; Sec. 6.1: the transmission calculation takes slant path
lengths at several altitudes, the optical depth and transmission along them,
multiplies by 2 pi r and integrates over altitude; the result is a transmission
modulation spectrum that the spectrum integrator bins into channels).
"""
from __future__ import annotations

import numpy as np

from .atmosphere import atmosphere, FLAG_T_CLAMP, FLAG_RADIUS
from .constants import C2, C_LIGHT, H_PLANCK


def interp_index(t_grid: np.ndarray, temp: float):
    """Linear-in-T interpolation bracket: k = largest index with T_k <= T, clamped to
    [0, NT-2]; weight w = (T - T_k)/(T_{k+1} - T_k) clamped to [0, 1].
    Returns (k, w, clamped)."""
    nt = t_grid.size
    k = int(np.searchsorted(t_grid, temp, side="right")) - 1
    k = min(max(k, 0), nt - 2)
    w = (temp - t_grid[k]) / (t_grid[k + 1] - t_grid[k])
    clamped = not (t_grid[0] <= temp <= t_grid[-1])
    w = min(max(w, 0.0), 1.0)
    return k, w, clamped


def extinction(sigma: np.ndarray, t_grid: np.ndarray, temp: np.ndarray, n_species: np.ndarray,
               cia: np.ndarray | None = None, cia_t_grid: np.ndarray | None = None,
               n_h2: np.ndarray | None = None, cia_he: np.ndarray | None = None,
               n_he: np.ndarray | None = None):
    """Step a3. sigma[S][NT][L][Nnu] in cm^2/molecule on the layer pressures;
    e_l(nu) = sum_i n_{i,l} sigma_i(T_l, p_l, nu)
              + n_{H2,l}^2 K(T_l, nu)            (H2-H2 CIA, cm^5 molecule^-2)
              + n_{H2,l} n_{He,l} K_He(T_l, nu)  (H2-He CIA, when given; Sec. 3 and the
                                                  HITRAN CIA source the paper cites)
    with sigma and the CIA coefficients interpolated linearly in T (both CIA tables on
    the same temperature grid). Returns (e[L][Nnu], flags)."""
    S, NT, L, NNU = sigma.shape
    e = np.zeros((L, NNU), dtype=np.float64)
    flags = 0
    for l in range(L):
        k, w, clamped = interp_index(t_grid, temp[l])
        if clamped:
            flags |= FLAG_T_CLAMP
        for i in range(S):
            s_lo = sigma[i, k, l].astype(np.float64)
            s_hi = sigma[i, k + 1, l].astype(np.float64)
            e[l] += n_species[i, l] * ((1.0 - w) * s_lo + w * s_hi)
        if cia is not None:
            kc, wc, clamped = interp_index(cia_t_grid, temp[l])
            if clamped:
                flags |= FLAG_T_CLAMP
            c_lo = cia[kc].astype(np.float64)
            c_hi = cia[kc + 1].astype(np.float64)
            e[l] += n_h2[l] ** 2 * ((1.0 - wc) * c_lo + wc * c_hi)
            if cia_he is not None:
                h_lo = cia_he[kc].astype(np.float64)
                h_hi = cia_he[kc + 1].astype(np.float64)
                e[l] += n_h2[l] * n_he[l] * ((1.0 - wc) * h_lo + wc * h_hi)
    return e, flags


def rayleigh_h2(nu: np.ndarray) -> np.ndarray:
    """H2 Rayleigh-scattering cross section (cm^2 molecule^-1) at wavenumbers nu (cm^-1),
    the Dalgarno & Williams (1962) expansion in the wavelength in Angstrom:
    sigma = 8.14e-13 lam^-4 + 1.28e-6 lam^-6 + 1.61 lam^-8 (Sec. 3: transit's Rayleigh
    scattering; the paper gives no formula, this is the standard one for H2)."""
    lam = 1.0e8 / np.asarray(nu, dtype=np.float64)
    return 8.14e-13 / lam ** 4 + 1.28e-6 / lam ** 6 + 1.61 / lam ** 8


def cloud_layer(p_bar: np.ndarray, log_p_cloud: float) -> int:
    """Gray cloud deck (Sec. 3; the cloud-top pressure of the Sec. 7 retrievals): the
    deepest-first index of the last layer at or below the cloud top, i.e. the largest l with
    p_l >= p_cloud (-1 when the deck lies below every layer). Chords whose impact parameter
    lies at or below that layer are opaque."""
    p_cloud = 10.0 ** log_p_cloud
    below = np.nonzero(np.asarray(p_bar) >= p_cloud)[0]
    return int(below.max()) if below.size else -1


def chord_path(radius: np.ndarray, j: int, l: int) -> float:
    """Half-chord length from the tangent point of impact parameter b_j = r_j to the
    sphere of radius r_l (l >= j): s = sqrt(r_l^2 - r_j^2), written as a product of a
    difference and a sum to avoid cancellation."""
    return float(np.sqrt((radius[l] - radius[j]) * (radius[l] + radius[j])))


def optical_depth(radius: np.ndarray, ext: np.ndarray) -> np.ndarray:
    """Step a4. Chord optical depth at impact parameter b_j = r_j: the trapezoid in path
    length along both halves of the chord,
    tau_j = sum_{l=j}^{L-2} (s_{j,l+1} - s_{j,l}) (e_l + e_{l+1}),  tau_{L-1} = 0."""
    L, NNU = ext.shape
    tau = np.zeros((L, NNU), dtype=np.float64)
    for j in range(L):
        for l in range(j, L - 1):
            ds = chord_path(radius, j, l + 1) - chord_path(radius, j, l)
            tau[j] += ds * (ext[l] + ext[l + 1])
    return tau


def transit_depth(radius: np.ndarray, tau: np.ndarray, rs_cm: float,
                  tau_max: float | None = None, cloud_index: int = -1) -> np.ndarray:
    """Step a5. Transit depth: an opaque disk inside the deepest layer plus the
    absorbed fraction of each annulus, trapezoid in impact parameter,
    depth = [r_0^2 + 2 int_{r_0}^{r_top} (1 - exp(-tau(b))) b db] / Rs^2
          = [r_0^2 + sum_j (r_{j+1} - r_j)(f_j r_j + f_{j+1} r_{j+1})] / Rs^2,
    f = 1 - exp(-tau).
    With an optical-depth limit (Sec. 4 item 7: calculate only down to a user-set optical
    depth at each wavenumber), the rays are followed from the top impact parameter down;
    at the first one whose optical depth reaches tau_max, it and every deeper one count as
    opaque, f = 1. A gray cloud deck makes the chords j <= cloud_index opaque too."""
    L, NNU = tau.shape
    f = -np.expm1(-tau)
    if cloud_index >= 0:
        f[: cloud_index + 1] = 1.0
    if tau_max is not None and tau_max > 0:
        reached = np.zeros(NNU, dtype=bool)
        for j in range(L - 1, -1, -1):
            reached |= tau[j] >= tau_max
            f[j] = np.where(reached, 1.0, f[j])
    acc = np.full(NNU, radius[0] ** 2, dtype=np.float64)
    for j in range(L - 1):
        acc += (radius[j + 1] - radius[j]) * (f[j] * radius[j] + f[j + 1] * radius[j + 1])
    return acc / rs_cm ** 2


def planck(nu: np.ndarray, temp: float) -> np.ndarray:
    """Planck function per unit wavenumber, B_nu(T) = 2 h c^2 nu^3 / (exp(c2 nu / T) - 1)
    in erg s^-1 cm^-2 sr^-1 (cm^-1)^-1, nu in cm^-1 (c2 = h c / k_B)."""
    nu = np.asarray(nu, dtype=np.float64)
    return 2.0 * H_PLANCK * C_LIGHT ** 2 * nu ** 3 / np.expm1(C2 * nu / temp)


def vertical_optical_depth(radius: np.ndarray, ext: np.ndarray) -> np.ndarray:
    """Emission (eclipse) geometry, plane-parallel layers at the hydrostatic radii:
    optical depth along the vertical from the top, trapezoid in height,
    tau_{L-1} = 0, tau_l = tau_{l+1} + (r_{l+1} - r_l)(e_l + e_{l+1}) / 2."""
    L, NNU = ext.shape
    tau = np.zeros((L, NNU), dtype=np.float64)
    for l in range(L - 2, -1, -1):
        tau[l] = tau[l + 1] + (radius[l + 1] - radius[l]) * 0.5 * (ext[l] + ext[l + 1])
    return tau


def emergent_intensity(temp: np.ndarray, tau: np.ndarray, nu: np.ndarray) -> np.ndarray:
    """Emission spectrum: the intensity emerging along the normal (the intensity spectra the
    paper's eclipse-geometry tests compare, Sec. 6), no scattering, the Planck function as
    source. The deepest layer radiates as a blackbody from below (no rays reach the abyss);
    between layers the source is the mean of the two layers' Planck functions:
    I = B(T_0) e^{-tau_0} + sum_l (B(T_l) + B(T_{l+1}))/2 (e^{-tau_{l+1}} - e^{-tau_l}).
    An isothermal atmosphere therefore emits exactly B(T) (the f08 test)."""
    L = tau.shape[0]
    b = np.array([planck(nu, float(t)) for t in temp])
    att = np.exp(-tau)
    out = b[0] * att[0]
    for l in range(L - 1):
        out = out + 0.5 * (b[l] + b[l + 1]) * (att[l + 1] - att[l])
    return out


def bin_spectrum(depth: np.ndarray, bin_width: int) -> np.ndarray:
    """Step a6 (spectrum integrator). Channels with perfect transmission over their
    range (Sec. 6.3): the mean of each group of ``bin_width`` consecutive points;
    a ragged tail shorter than a bin is dropped."""
    nb = depth.size // bin_width
    return depth[: nb * bin_width].reshape(nb, bin_width).mean(axis=1)


def chi_squared(model: np.ndarray, data: np.ndarray, err: np.ndarray) -> float:
    """Step a6. chi^2 = sum ((model - data) / err)^2 (Sec. 3: MC3 computes chi^2)."""
    return float(np.sum(((model - data) / err) ** 2))


def forward(params: np.ndarray, setup, sigma: np.ndarray, cia: np.ndarray | None = None,
            data: np.ndarray | None = None, err: np.ndarray | None = None,
            cia_he: np.ndarray | None = None):
    """Steps a1-a6 for one parameter vector. Returns a dict with the spectrum, the
    intermediate arrays, binned depths and chi^2 (when data are given), and flags.
    A sample whose radii are invalid gets a NaN spectrum. With setup.geometry == "eclipse"
    the spectrum (key "depth") is the emergent intensity instead of the transit depth."""
    atm = atmosphere(params, setup.p_bar, setup.mass_amu, setup.tp_mode, setup.planet)
    flags = atm["flags"]
    ext, f = extinction(sigma, setup.temps, atm["temp"], atm["n_species"],
                        cia, setup.cia_temps, atm["n_h2"], cia_he, atm["n_he"])
    flags |= f
    if getattr(setup, "rayleigh", False):
        ext = ext + atm["n_h2"][:, None] * rayleigh_h2(setup.nu)[None, :]
    jc = -1
    if getattr(setup, "cloud", False):
        jc = cloud_layer(setup.p_bar, float(params[-1]))
    if flags & FLAG_RADIUS:
        nan = np.full(setup.nu.size, np.nan)
        out = dict(atm=atm, ext=ext, tau=None, depth=nan, flags=flags)
    elif getattr(setup, "geometry", "transit") == "eclipse":
        tau = vertical_optical_depth(atm["radius"], ext)
        out = dict(atm=atm, ext=ext, tau=tau, depth=emergent_intensity(atm["temp"], tau, setup.nu),
                   flags=flags)
    else:
        tau = optical_depth(atm["radius"], ext)
        depth = transit_depth(atm["radius"], tau, setup.planet.rs_cm,
                              getattr(setup, "tau_max", None), jc)
        out = dict(atm=atm, ext=ext, tau=tau, depth=depth, flags=flags)
    if setup.bin_width:
        out["binned"] = bin_spectrum(out["depth"], setup.bin_width)
        if data is not None:
            out["chi2"] = chi_squared(out["binned"], data, err)
    return out
