"""Units and constants of the oracle (CODATA 2018).

Energies in eV, lengths in Angstrom, masses in amu, temperature in K and time in
fs.  Phonon "frequencies" are carried as energies hbar*omega in eV.
"""
import math

HBAR_EV_FS = 0.6582119569             # hbar in eV*fs
KB_EV = 8.617333262e-5                 # Boltzmann constant, eV/K
HBAR2_AMU_A2 = 0.004180159280496722    # hbar^2/(amu*Angstrom^2) in eV
E2_4PIEPS0 = 14.3996454784             # e^2/(4 pi eps_0), eV*Angstrom
TWO_PI = 2.0 * math.pi
SQRT_PI = math.sqrt(math.pi)
