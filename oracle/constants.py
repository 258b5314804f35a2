"""Physical constants in CGS (oracle copy; the GPU library keeps its own)."""
C_LIGHT = 2.99792458e10          # cm / s
K_BOLTZ = 1.380649e-16           # erg / K
H_PLANCK = 6.62607015e-27        # erg s
EV_ERG = 1.602176634e-12         # erg / eV
M_H = 1.6735575e-24              # g, hydrogen atom
M_E = 9.1093837015e-28           # g, electron
SIGMA_T = 6.6524587321e-25       # cm^2, Thomson
A_RAD = 7.565723e-15             # erg cm^-3 K^-4, radiation constant
T_CMB0 = 2.725                   # K, CMB temperature today
KPC_CM = 3.0856775814913673e21   # cm
MPC_CM = 3.0856775814913673e24   # cm
MYR_S = 3.15576e13               # s (Julian year)
H100_S = 1.0e7 / MPC_CM          # 100 km/s/Mpc in 1/s
GAMMA_ADIABATIC = 5.0 / 3.0      # ratio of specific heats (paper: 5/3)

__all__ = [n for n in dir() if n.isupper()]
