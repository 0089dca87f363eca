"""Closed-form reference solutions used by the physics checks (test infrastructure; no method
arithmetic: these are textbook flows, not the lattice Boltzmann step).

Layered channel: steady two-layer Poiseuille flow between no-slip walls at y' = 0 and y' = L
(the half-way walls half a node outside the first and last rows), driven by a uniform body
force G along x.  The shear stress nu u' = C - G y' is linear across the channel (Stokes flow,
stress continuity) and u(0) = u(L) = 0 fixes C.
"""
import math

import numpy as np


def diffuse_poiseuille(L, nu1, nu2, G, W):
    """Profile for the diffuse viscosity profile the method actually has: phi = tanh((L/2 - y')/W)
    and omega interpolated linearly in phi between omega(nu1) at phi = +1 and omega(nu2) at
    phi = -1 (nu = (1/omega - 1/2)/3), evaluated at the node centres y' = j + 1/2."""
    from scipy.integrate import quad

    wl, wg = 1 / (3 * nu1 + 0.5), 1 / (3 * nu2 + 0.5)

    def nu(s):
        ph = math.tanh((L / 2 - s) / W)
        w = wg + 0.5 * (ph + 1) * (wl - wg)
        return (1 / w - 0.5) / 3

    I0 = quad(lambda s: 1 / nu(s), 0, L, points=[L / 2], limit=200)[0]
    I1 = quad(lambda s: s / nu(s), 0, L, points=[L / 2], limit=200)[0]
    C = G * I1 / I0
    yp = np.arange(L) + 0.5
    return np.array([quad(lambda s: (C - G * s) / nu(s), 0, y, limit=200)[0] for y in yp])


def sharp_poiseuille(L, nu1, nu2, G):
    """Sharp-interface two-layer profile, interface at h = L/2 (nu1 below, nu2 above)."""
    h = L / 2
    C = G * (h * h / nu1 + (L * L - h * h) / nu2) / (2 * (h / nu1 + (L - h) / nu2))
    yp = np.arange(L) + 0.5
    return np.where(yp <= h, (C * yp - G * yp ** 2 / 2) / nu1, (G * (L * L - yp ** 2) / 2 - C * (L - yp)) / nu2)
