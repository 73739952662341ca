"""Physical constants and unit conversions (atomic units: hbar = m_e = e = 1).

The paper works in atomic units with hbar = 1 (Theory section, the light-matter
Hamiltonian in mass-weighted coordinates). These are the CODATA-style
conversions used to turn the workload description (Angstrom, fs, cm^-1, K, amu)
into atomic units. They are plain data: no step of the method lives here.
"""

ANGSTROM = 1.8897261246          # bohr per Angstrom
FS = 41.341373336                # atomic time units per femtosecond
HARTREE_CM = 219474.6313632      # cm^-1 per hartree
KB = 3.166811563e-6              # hartree per kelvin
C_AU = 137.035999084             # speed of light in a.u.
AMU = 1822.888486                # electron masses per unified atomic mass unit
MICRON = 1.0e4 * ANGSTROM        # bohr per micrometre

MASS_AMU = (15.999, 1.008)       # species 0 = O, 1 = H
SPECIES_NAMES = ("O", "H")
