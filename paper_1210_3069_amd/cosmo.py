"""Comoving distances for placing lens planes and galaxies (host side).

chi(a) = c int_a^1 da' / (a'^2 H(a')) with H(a) = H0 sqrt(Om a^-3 + 1 - Om)
for flat LCDM (Sec. 2.1), in h^-1 Mpc (c/H0 = 2997.92458 h^-1 Mpc).  The
integral is tabulated once with the trapezoid rule on a fine grid in a and
interpolated."""
import numpy as np

C_OVER_H0 = 2997.92458


def chi_of_z(z, omega_m=0.3, zmax=10.0, ngrid=200001):
    z = np.asarray(z, dtype=np.float64)
    a = np.linspace(1.0 / (1.0 + zmax), 1.0, ngrid)
    f = 1.0 / (a * a * np.sqrt(omega_m / a ** 3 + 1.0 - omega_m))
    # cumulative integral from a to 1
    seg = 0.5 * (f[1:] + f[:-1]) * np.diff(a)
    tail = np.concatenate([np.cumsum(seg[::-1])[::-1], [0.0]])
    return C_OVER_H0 * np.interp(1.0 / (1.0 + z), a, tail)
