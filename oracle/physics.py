"""Physical constants, species, argon cross sections and null-collision bounds.

Test infrastructure only (see ``oracle/__init__.py``).

The paper simulates helium with tabulated cross sections (Section 2b).  Those
tables are not available here, so the discharge is argon with the analytic
cross sections below (a builder-defined reading, fitted to no dataset):

* electron elastic       sigma_el = 1.0e-19 / (1 + eps/20)              m^2
* electron excitation    sigma_ex = 2.7e-20 ln(x)/x,  x = eps/11.5 > 1
* electron ionisation    sigma_iz = 7.6e-20 ln(x)/x,  x = eps/15.76 > 1
* ion charge exchange    sigma_cx = 5.0e-19 (constant)

with eps the electron energy in eV.  The null-collision bounds nu_max follow
Vahedi & Surendra (cited in Section 2): the electron bound is the maximum over
energy of n_g sum_p sigma_p(eps) v(eps) times a 2 % margin; the ion bound uses
the largest relative speed g_max = sqrt(4 e V0 / M) + 6 sqrt(k_B T_g / M).
"""
from __future__ import annotations

import math

import numpy as np

# CODATA 2018 values (e and k_B exact in the 2019 SI).
QE = 1.602176634e-19      # C
ME = 9.1093837015e-31     # kg
AMU = 1.66053906660e-27   # kg
EPS0 = 8.8541878128e-12   # F/m
KB = 1.380649e-23         # J/K
M_AR = 39.948 * AMU       # kg

# Species index -> (charge, mass).  0: electrons, 1: Ar+.
SPECIES = ((-QE, ME), (QE, M_AR))

E_EXC = 11.5     # eV, excitation threshold
E_ION = 15.76    # eV, ionisation threshold
SIGMA_CX = 5.0e-19

# Derived constants used in the collision arithmetic (formed the same way on
# both sides of the parity tests).
HALF_ME_OVER_QE = (0.5 * ME) / QE        # eps[eV] = HALF_ME_OVER_QE * |v|^2
TWO_QE_OVER_ME = (2.0 * QE) / ME         # |v|^2 = TWO_QE_OVER_ME * eps[eV]
TWO_ME_OVER_M = (2.0 * ME) / M_AR        # elastic energy-loss factor


def sigma_el(eps):
    return 1.0e-19 / (1.0 + eps / 20.0)


def _lnx_over_x(eps, thr, amp):
    eps = np.asarray(eps, dtype=np.float64)
    x = eps / thr
    out = np.zeros_like(x)
    m = eps > thr
    out[m] = amp * np.log(x[m]) / x[m]
    return out


def sigma_ex(eps):
    return _lnx_over_x(eps, E_EXC, 2.7e-20)


def sigma_iz(eps):
    return _lnx_over_x(eps, E_ION, 7.6e-20)


def gas_density(p_pa, t_gas_k):
    """n_g = p / (k_B T_g)."""
    return p_pa / (KB * t_gas_k)


def nu_max_electron(n_g):
    """Null-collision bound for electrons: 1.02 n_g max_eps sum_p sigma_p v.

    The maximum is taken on a log-spaced energy scan from 1e-3 eV to 1e5 eV;
    above ~64 eV the summed rate only decays, so the scan range bounds all
    energies.
    """
    eps = np.logspace(-3, 5, 200001)
    v = np.sqrt(TWO_QE_OVER_ME * eps)
    rate = (sigma_el(eps) + sigma_ex(eps) + sigma_iz(eps)) * v
    return 1.02 * n_g * float(rate.max())


def nu_max_ion(n_g, v0, t_gas_k):
    """Charge-exchange bound: n_g sigma_cx g_max."""
    g_max = math.sqrt(4.0 * QE * abs(v0) / M_AR) + 6.0 * math.sqrt(KB * t_gas_k / M_AR)
    return n_g * SIGMA_CX * g_max
