"""Shared builders for GPU tests: synthetic setups and their oracle / GPU views."""
from __future__ import annotations

import numpy as np

import workloads as wl


def small_config2(n_nu=1000, n_layers=100, seed=11, dnu=0.5):
    """Config-2 shapes (4 absorbers, 20 T, five-parameter T(p), CIA, 30-point bins)
    with a random opacity table; Nnu reduced so the oracle runs in well under a second."""
    s = wl.config2(n_nu=n_nu, n_layers=n_layers, dnu=dnu)
    sigma = wl.random_opacity_table(s.n_species, s.temps, n_layers, s.nu, seed=seed,
                                    dtype=np.float32)
    cia = wl.cia_table(s.cia_temps, s.nu)
    return s, sigma, cia


def config1_table(n_nu=1000, seed=12):
    s = wl.config1()
    if n_nu != s.nu.size:
        s.nu = s.nu[:n_nu]
    sigma = wl.random_opacity_table(1, s.temps, s.p_bar.size, s.nu, seed=seed)
    return s, sigma


def gpu_model(setup, sigma, cia=None, data=None, err=None, device="cuda", cia_he=None, tiles=True):
    import torch
    import paper_2104_12522_amd as bm
    return bm.Model(torch.as_tensor(sigma), setup.temps, setup.p_bar, setup.mass_amu,
                    setup.tp_mode, setup.planet,
                    cia=None if cia is None else torch.as_tensor(cia),
                    cia_temps=setup.cia_temps if cia is not None else None,
                    bin_width=setup.bin_width, data=data, err=err, device=device,
                    tau_max=setup.tau_max, nu_start=float(setup.nu[0]),
                    dnu=float(setup.nu[1] - setup.nu[0]) if setup.nu.size > 1 else 1.0,
                    rayleigh=setup.rayleigh, cloud=setup.cloud, geometry=setup.geometry,
                    cia_he=None if cia_he is None else torch.as_tensor(cia_he), tiles=tiles)


def prior_for(setup):
    p = (wl.isothermal_prior(setup.n_species) if setup.tp_mode == 0
         else wl.line2013_prior(setup.n_species))
    return wl.with_cloud(p) if setup.cloud else p
