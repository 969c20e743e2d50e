"""Linear kinetic dispersion relation of a 1D electrostatic electron plasma
with immobile ions (textbook result, not from the paper):

    1 + sum_s w_s / k^2 * [1 + zeta_s Z(zeta_s)] = 0,
    zeta_s = (omega - k u_s) / (k sqrt(2)),  Z(z) = i sqrt(pi) w(z)

for Maxwellian beams of unit thermal speed, drift u_s and weight w_s.  Used
by the tests to pin the oracle's Landau damping and two-stream growth rates.
"""
import numpy as np
from scipy.optimize import fsolve
from scipy.special import wofz


def dispersion(omega, k, beams):
    eps = 1.0 + 0j
    for w, u in beams:
        z = (omega - k * u) / (k * np.sqrt(2.0))
        Z = 1j * np.sqrt(np.pi) * wofz(z)
        eps += w / k ** 2 * (1.0 + z * Z)
    return eps


def root(k, beams, guess):
    def f(xy):
        e = dispersion(xy[0] + 1j * xy[1], k, beams)
        return [e.real, e.imag]
    x, y = fsolve(f, [guess.real, guess.imag], xtol=1e-13)
    return complex(x, y)


def fit_rate(t, W, t0, t1, peaks=True):
    """Slope/2 of log W over [t0, t1]; with peaks=True only local maxima
    are fitted (oscillating field energy)."""
    t = np.asarray(t)
    W = np.asarray(W)
    sel = (t >= t0) & (t <= t1)
    if peaks:
        idx = [i for i in range(1, len(W) - 1)
               if W[i] >= W[i - 1] and W[i] >= W[i + 1] and sel[i]]
        tt, ww = t[idx], W[idx]
    else:
        tt, ww = t[sel], W[sel]
    slope = np.polyfit(tt, np.log(ww), 1)[0]
    return 0.5 * slope, tt


def dispersion_species(omega, k, species):
    """1 + sum_s wp2_s / (k vth_s)^2 [1 + zeta_s Z(zeta_s)], zeta_s =
    (omega - k u_s) / (sqrt(2) k vth_s), for species (wp2, vth, u)."""
    eps = 1.0 + 0j
    for wp2, vth, u in species:
        z = (omega - k * u) / (np.sqrt(2.0) * k * vth)
        Z = 1j * np.sqrt(np.pi) * wofz(z)
        eps += wp2 / (k * vth) ** 2 * (1.0 + z * Z)
    return eps


def root_species(k, species, guess):
    def f(xy):
        e = dispersion_species(xy[0] + 1j * xy[1], k, species)
        return [e.real, e.imag]
    x, y = fsolve(f, [guess.real, guess.imag], xtol=1e-13)
    return complex(x, y)
