"""Constants of the method, each with the passage that fixes it.

Test infrastructure (see the package docstring): not shared with the GPU path.
"""

# AB flux zero-point for a source at 10 pc, in L_sun/Hz (Section 2.2.1,
# definition after Eq. restmag).
AB0_LSUN_PER_HZ = 1.13492e-13

# Reference V-band wavelength of the attenuation power law (Section 3.4,
# after Eq. salim): 5500 Angstrom.
LAMBDA_V_ANGSTROM = 5500.0

# Normalisation of the attenuation curve, A_lambda = A_V / 4.05 * k_lambda
# (Section 3.4, Eq. salim).
R_V_SALIM = 4.05

# Switch between the two k0 branches (Section 3.4, Eq. kzero): 0.15 micron.
K0_SWITCH_MICRON = 0.15

# Drude bump width and centre (Section 3.4, Eq. uvbump and the text after it).
DRUDE_WIDTH_ANGSTROM = 350.0
DRUDE_CENTRE_ANGSTROM = 2175.0

# Speed of light in km/s and the Hubble time unit: 1/H0 in Gyr equals
# HUBBLE_TIME_GYR_KMS_MPC / H0 with H0 in km/s/Mpc (Julian year, IAU parsec).
C_KM_S = 299792.458
HUBBLE_TIME_GYR_KMS_MPC = 977.7922216807891

# Years per Gyr: the SFR is in M_sun/yr and the time grid in Gyr.
YR_PER_GYR = 1.0e9

# Width of the quenching transition in the parametric SFH stand-in, in Gyr.
SFH_QUENCH_WIDTH_GYR = 0.5
