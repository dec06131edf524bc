"""Fluid and rock properties for the synthetic thermal multiphase problems.

Every function is written with numpy operations that are complex-analytic in
their arguments, so that the Jacobian can be formed by complex-step
differentiation (derivatives exact to rounding).

Sources for the correlations and constants:
  * water viscosity: Grabowski correlation, Appendix A (eq:watermu, tab:watermu);
  * water density: Trangenstein's modification of Kell's formula, Appendix A
    (tab:waterrho); temperature in degC and pressure in MPa;
  * relative permeabilities k_ra = S_a, Appendix A;
  * rock and fluid heat constants, initial pressure: tab:parameters (Section 4).
The oil viscosity / density constants and the gas phase are not given in the
paper (they are deferred to the companion paper); the values below are the
synthetic choices documented with the design notes.
"""
import numpy as np

# ---- tab:parameters (Section 4) -------------------------------------------
P_INIT = 4.1369e7          # Pa
K_T_OIL = 0.15             # W/(m K)
K_T_WATER = 0.6005638      # W/(m K)
K_T_ROCK = 1.7295772056    # W/(m K)
CV_OIL = 2093.4            # J/(K kg)
CV_WATER = 4181.3          # J/(K kg)
CV_ROCK = 920.0            # J/(K kg)
RHO_ROCK = 2650.0          # kg/m^3 (printed unit is garbled; m^-3 is meant)

# ---- initial state / scaling (Section 4: 60 F initial temperature of the
# SPE10-style cases, So = 0.9 of the refinement study) --------------------
T_INIT = 288.706           # K
T_INJ = 373.15             # K, hot water injection temperature
T_HEATER = 373.15          # K
G = 9.80665                # m/s^2, along -z
P_BHP = 2.7579e7           # Pa, producer bottom-hole pressure (SPE10 case)

# ---- synthetic choices (not in the paper) --------------------------------
MU_O_REF = 10.0            # Pa s (1e4 cP) at T_INIT
MU_O_B = 7400.0            # K, Arrhenius coefficient of the oil viscosity
RHO_O_SURF = 999.0         # kg/m^3, API 10 => equal to water at surface
C_OIL = 1.0e-9             # 1/Pa, oil compressibility
BETA_OIL = 4.0e-4          # 1/K, oil thermal expansion
P_SURF = 1.01325e5         # Pa
GAS_M = 0.016              # kg/mol (methane)
GAS_R = 8.314462618        # J/(mol K)
MU_GAS = 1.5e-5            # Pa s
CV_GAS = 1700.0            # J/(K kg)
K_T_GAS = 0.03             # W/(m K)
HEATER_U = 1.0e3           # W/K per heated cell
Q_INJ = 1.0e-7             # m^3/s of water per completed injector cell
WELL_RW = 0.01             # m, wellbore radius of the Peaceman producer

# ---- Appendix A tables ---------------------------------------------------
GRAB_A, GRAB_B, GRAB_C = 2.1850, 0.04012, 5.1547e-6
KELL_E = (999.83952, 16.955176, -7.987e-3, -46.170461e-6, 105.56302e-9,
          -280.54353e-12)
KELL_E6 = 16.87985e-3
KELL_E7 = 10.2             # MPa
KELL_CW = 3.98854e-4       # 1/MPa


def mu_water(T):
    """Grabowski water viscosity (Appendix A): argument in K, result in Pa s."""
    tf = (T - 273.15) * 1.8 + 32.0
    return 1.0e-3 * GRAB_A / (-1.0 + GRAB_B * tf + GRAB_C * tf * tf)


def rho_water(p, T):
    """Kell/Trangenstein water density (Appendix A), degC and MPa inside."""
    tc = T - 273.15
    e0, e1, e2, e3, e4, e5 = KELL_E
    num = e0 + tc * (e1 + tc * (e2 + tc * (e3 + tc * (e4 + tc * e5))))
    return num / (1.0 + KELL_E6 * tc) * np.exp(KELL_CW * (p * 1.0e-6 - KELL_E7))


def mu_oil(T):
    """Heavy-oil viscosity, Arrhenius form (synthetic constants)."""
    return MU_O_REF * np.exp(MU_O_B * (1.0 / T - 1.0 / T_INIT))


def rho_oil(p, T):
    """Exponential oil density correlation (synthetic constants)."""
    return RHO_O_SURF * np.exp(C_OIL * (p - P_SURF) - BETA_OIL * (T - T_INIT))


def mu_gas(T):
    return MU_GAS + 0.0 * T


def rho_gas(p, T):
    """Ideal gas density p M / (R T)."""
    return p * GAS_M / (GAS_R * T)


class Phase:
    def __init__(self, name, rho, mu, cv, k_t):
        self.name, self.rho, self.mu, self.cv, self.k_t = name, rho, mu, cv, k_t


WATER = Phase("w", rho_water, mu_water, CV_WATER, K_T_WATER)
OIL = Phase("o", rho_oil, mu_oil, CV_OIL, K_T_OIL)
GAS = Phase("g", rho_gas, mu_gas, CV_GAS, K_T_GAS)


def frozen_T(phase, T0=T_INIT):
    """Copy of a phase whose density and viscosity ignore temperature.

    With such phases the assembled Schur approximation equals the exact
    A_TT block (compare the A_TT expression of Section 3 with eq:Se)."""
    return Phase(phase.name + "*", lambda p, T: phase.rho(p, T0 + 0.0 * T),
                 lambda T: phase.mu(T0 + 0.0 * T), phase.cv, phase.k_t)
