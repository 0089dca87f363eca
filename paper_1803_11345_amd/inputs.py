"""Seeded synthetic initial states for the lattice Boltzmann step.

This module holds no arithmetic of the method itself: it only builds the initial order
parameter, density and velocity planes (float64, shape (ny, nx), x fastest) that both the
GPU path and the CPU oracle start from.  Random numbers come from SplitMix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014), evaluated counter-style:
value k of stream ``seed`` is the SplitMix64 output for state seed + (k + 1) * golden gamma, so
a row-major fill is reproducible in any language.
"""
from __future__ import annotations

import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Outputs offset .. offset+count-1 of the SplitMix64 sequence started at ``seed``."""
    with np.errstate(over="ignore"):
        k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = np.uint64(seed) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform(seed: int, count: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """``count`` doubles uniform in [lo, hi) from the top 53 bits of SplitMix64."""
    u = (splitmix64(seed, count) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return lo + (hi - lo) * u


def interface_width(a: float, gamma: float) -> float:
    """Width W of the equilibrium profile phi = tanh(d / W): W = sqrt(2 gamma / a)."""
    return math.sqrt(2.0 * gamma / a)


def droplet(nx: int, ny: int, radius: float, width: float, cx: float | None = None,
            cy: float | None = None) -> np.ndarray:
    """phi = tanh((R - r) / W) around (cx, cy) (default: the lattice centre nx/2, ny/2),
    positive inside.  Distances are taken in node-index coordinates without periodic images."""
    cx = nx / 2.0 if cx is None else cx
    cy = ny / 2.0 if cy is None else cy
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.hypot(x - cx, y - cy)
    return np.tanh((radius - r) / width)


def layered(nx: int, ny: int, width: float, y_interface: float | None = None) -> np.ndarray:
    """phi = +1 below ``y_interface`` (default (ny - 1) / 2, mid-channel between walls at
    y = -1/2 and y = ny - 1/2) and -1 above, joined by tanh((y_i - y) / W)."""
    yi = (ny - 1) / 2.0 if y_interface is None else y_interface
    y = np.arange(ny, dtype=np.float64)
    col = np.tanh((yi - y) / width)
    return np.repeat(col[:, None], nx, axis=1)


def band(nx: int, ny: int, width: float, y_lo: float, y_hi: float) -> np.ndarray:
    """A periodic flat band: phi = +1 for y_lo < y < y_hi, -1 outside, two tanh interfaces."""
    y = np.arange(ny, dtype=np.float64)
    col = np.tanh((y - y_lo) / width) - np.tanh((y - y_hi) / width) - 1.0
    return np.repeat(col[:, None], nx, axis=1)


def spinodal(nx: int, ny: int, seed: int = 1, amplitude: float = 0.05) -> np.ndarray:
    """phi i.i.d. uniform in [-amplitude, amplitude), row-major fill from SplitMix64(seed)."""
    return uniform(seed, nx * ny, -amplitude, amplitude).reshape(ny, nx)


def smooth_state(nx: int, ny: int, seed: int, u_amp: float = 0.05, rho_amp: float = 0.02,
                 modes: int = 3, interfaces: bool = True):
    """A random smooth periodic state (phi, rho, ux, uy), built from a few Fourier modes with
    SplitMix64 amplitudes and phases.  With ``interfaces`` phi is tanh-compressed so that it
    spans both phases with diffuse interfaces a few nodes wide."""
    r = uniform(seed, 6 * 4 * modes * modes, -1.0, 1.0).reshape(6, 4, modes, modes)
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)

    def field(k):
        out = np.zeros((ny, nx))
        for m in range(modes):
            for n in range(modes):
                kx = 2 * math.pi * m / nx
                ky = 2 * math.pi * n / ny
                amp = r[k, 0, m, n] / (1.0 + m + n)
                ph = math.pi * r[k, 1, m, n]
                out += amp * np.cos(kx * x + ky * y + ph)
                amp2 = r[k, 2, m, n] / (1.0 + m + n)
                out += amp2 * np.sin(kx * x - ky * y + math.pi * r[k, 3, m, n])
        s = np.max(np.abs(out))
        return out / s if s > 0 else out

    phi = field(0)
    if interfaces:
        phi = np.tanh(3.0 * phi)
    rho = 1.0 + rho_amp * field(1)
    ux = u_amp * field(2)
    uy = u_amp * field(3)
    return phi, rho, ux, uy


def ensemble(count: int, seed: int = 7, sides=(64, 128, 256, 512, 1024), a: float = 0.04,
             gamma: float = 0.04, nu1: float = 0.1, force: float = 1e-6):
    """A seeded ensemble of independent square boxes: side uniform over ``sides``; each box a
    static droplet (periodic, R uniform in [0.15, 0.35] * side, nu_l = nu1, nu_g = nu1 / ratio) or
    a layered channel (walls in y, body force along x, phi = +1 below with nu1 and -1 above with
    ratio * nu1), with the viscosity ratio log-uniform in [1, 1000].  The default a = gamma = 0.04
    are the free-energy constants of the paper's high-contrast bubble runs.  Returns a list of
    (params, phi0) with params a dict of lattice parameters."""
    u = uniform(seed, 4 * count).reshape(count, 4)
    W = interface_width(a, gamma)
    out = []
    for k in range(count):
        side = int(sides[min(int(u[k, 0] * len(sides)), len(sides) - 1)])
        ratio = 10.0 ** (3.0 * u[k, 2])
        if u[k, 1] < 0.5:
            radius = (0.15 + 0.2 * u[k, 3]) * side
            params = dict(nx=side, ny=side, bc_y=0, a=a, gamma=gamma, nu_l=nu1, nu_g=nu1 / ratio)
            phi0 = droplet(side, side, radius, W)
        else:
            params = dict(nx=side, ny=side, bc_y=1, a=a, gamma=gamma, nu_l=nu1, nu_g=nu1 * ratio,
                          force_x=force)
            phi0 = layered(side, side, W)
        out.append((params, phi0))
    return out


def two_droplets(nx: int, ny: int, r1: float, r2: float, gap: float, width: float) -> np.ndarray:
    """Two droplets side by side along x, centred in the box, whose surfaces are ``gap`` nodes
    apart: phi = tanh((r1 - d1) / W) + tanh((r2 - d2) / W) + 1 (+1 inside either, -1 outside)."""
    span = 2 * r1 + gap + 2 * r2
    x0 = nx / 2.0 - span / 2.0
    c1, c2 = x0 + r1, x0 + 2 * r1 + gap + r2
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    d1 = np.hypot(x - c1, y - ny / 2.0)
    d2 = np.hypot(x - c2, y - ny / 2.0)
    return np.tanh((r1 - d1) / width) + np.tanh((r2 - d2) / width) + 1.0


def coalescence_cases(count: int, seed: int = 11, rmin: float = 20.0, rmax: float = 40.0, gmin: float = 2.0,
                      gmax: float = 6.0):
    """``count`` (r1, r2, gap) triples: radii uniform in [rmin, rmax], gap uniform in [gmin, gmax]."""
    u = uniform(seed, 3 * count).reshape(count, 3)
    return [(rmin + (rmax - rmin) * a, rmin + (rmax - rmin) * b, gmin + (gmax - gmin) * c) for a, b, c in u]


def he_uniform(seed: int, shapes):
    """Seeded initial network parameters: for each (fan_in, count, zero) entry, ``count`` values
    uniform in +-sqrt(6 / fan_in) (He et al., ICCV 2015, uniform form), or zeros when ``zero``."""
    out = []
    for k, (fan_in, count, zero) in enumerate(shapes):
        if zero:
            out.append(np.zeros(count))
        else:
            lim = math.sqrt(6.0 / fan_in)
            out.append(uniform(seed * 1000 + k, count, -lim, lim))
    return np.concatenate(out) if out else np.zeros(0)
