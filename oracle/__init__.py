"""Plain FP64 CPU oracle for the BART transmission forward model.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports, calls or links
anything here; only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` do. It shares no code with the GPU library: it is written
from the paper (Harrington et al., "BART I", arXiv:2104.12522) and from the
readings listed below, in numpy/scipy float64, without blocking, fusion or
reordering beyond what each definition states.

Modules
-------
constants   physical constants (CGS)
atmosphere  T(p) profiles, composition, number densities, hydrostatic radii
rt          temperature interpolation, extinction, chord optical depth,
            transit depth, band binning, chi-squared, full forward model
opacity     line strengths, widths, Voigt profile, brute-force opacity table
stats       SPEIS / ESS / credible-region error (Sec. 5, App. C), Gelman-Rubin
mcmc        reference DE-MCz sampler and delayed acceptance
mlp         FP64 multilayer perceptron forward / backward / Adam

Readings of the paper (where it is silent the oracle follows these):
 * T interpolation is linear in T, clamped to the table, and flagged when clamped.
 * The chord and impact-parameter integrals are trapezoids in path length and in
   impact parameter, with impact parameters at the layer radii and an opaque disk
   inside the deepest layer.
 * Hydrostatic radii use g = GM/r^2 and the exact integral of the piecewise-linear
   (in ln p) temperature profile, anchored at the reference pressure.
 * The five-parameter T(p) profile is the one of Line et al. (2013), which the paper
   cites for its retrievals (Sec. 6.3, Sec. 7).
 * Filler gas is H2:He = 0.85:0.15 (Table 1, the Barstow et al. models).
 * Line strengths scale with a power-law partition function Q ~ T^1.5, Lorentz widths
   scale as (p / 1 atm) (296/T)^0.5, the Doppler width is the Gaussian standard
   deviation of Eq. 2, and the 25-HWHM cutoff uses the Voigt HWHM of Olivero &
   Longbothum (1977).
"""
