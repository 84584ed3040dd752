"""Physical constants in CGS units (oracle side; test infrastructure only)."""
K_B = 1.380649e-16          # erg / K
M_U = 1.66053906660e-24     # g (atomic mass unit)
C_LIGHT = 2.99792458e10     # cm / s
C2 = 1.4387769              # h c / k_B, cm K
G_GRAV = 6.67430e-8         # cm^3 g^-1 s^-2
BAR = 1.0e6                 # dyn / cm^2
ATM_BAR = 1.01325           # 1 atm in bar
T_REF = 296.0               # line-list reference temperature, K
H_PLANCK = 6.62607015e-27     # erg s
