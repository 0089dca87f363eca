"""FP64 CPU oracle of the hybrid central-moments / BGK lattice Boltzmann step
(arXiv:1803.11345), wrapped with ctypes.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg of the
benchmark are the only callers.  The GPU library never imports, links or executes anything
in this package, and this package imports nothing from the GPU library.

The C source (``lbcm_oracle.c``) holds the arithmetic; this module only marshals numpy arrays.
Population arrays have shape (9, ny, nx), float64, C order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbcm_oracle.c")
_LIB = os.path.join(_HERE, "liblbcm_oracle.so")


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (-O3 for the x86-64-v3 level (AVX2, FMA units), OpenMP).
    Floating-point contraction stays off and no fast-math option is given, so every operation
    rounds as written in the source: the results are those of any IEEE double build.  Always
    recompiles."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-o", tmp, _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


@dataclass
class Params:
    """Mirror of ``orc_params``: lattice size, boundary kind and the physical constants."""

    nx: int
    ny: int
    walls: int = 0
    a: float = 0.04
    gamma: float = 0.08
    mobility: float = 0.1
    Gamma: float = 1.0
    nu_l: float = 1.0 / 6.0
    nu_g: float = 1.0 / 6.0
    omega3: float = 1.0
    force_x: float = 0.0
    force_y: float = 0.0
    wall_ux_bottom: float = 0.0
    wall_ux_top: float = 0.0
    wall_gradient: float = 0.0
    k8_printed: int = 0
    collision: int = 0
    nthreads: int = 0


class _CParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("walls", ctypes.c_int),
        ("a", ctypes.c_double), ("gamma", ctypes.c_double), ("mobility", ctypes.c_double),
        ("Gamma", ctypes.c_double), ("nu_l", ctypes.c_double), ("nu_g", ctypes.c_double),
        ("omega3", ctypes.c_double), ("force_x", ctypes.c_double), ("force_y", ctypes.c_double),
        ("wall_ux_bottom", ctypes.c_double), ("wall_ux_top", ctypes.c_double), ("wall_gradient", ctypes.c_double),
        ("k8_printed", ctypes.c_int), ("collision", ctypes.c_int), ("nthreads", ctypes.c_int),
    ]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_CParams)
        d = ctypes.c_double
        lib.orc_check.argtypes = [P]
        lib.orc_stencil.argtypes = [P, _D, _D, _D, _D]
        lib.orc_stencil.restype = None
        lib.orc_feq.argtypes = [d, d, d, d, d, d, d, _D]
        lib.orc_feq.restype = None
        lib.orc_geq.argtypes = [d, d, d, d, d, _D]
        lib.orc_geq.restype = None
        lib.orc_tmatrix.argtypes = [d, d, _D]
        lib.orc_tmatrix.restype = None
        lib.orc_keq.argtypes = [d, d, d, d, d, d, d, d, ctypes.c_int, _D]
        lib.orc_keq.restype = None
        lib.orc_guo.argtypes = [d, d, d, d, _D]
        lib.orc_guo.restype = None
        lib.orc_collide_f.argtypes = [P, _D, d, d, d, d, _D, _D]
        lib.orc_collide_f.restype = None
        lib.orc_collide_g.argtypes = [P, _D, d, d, d, d, _D]
        lib.orc_collide_g.restype = None
        for name in ("orc_mu", "orc_p0", "orc_ptilde"):
            getattr(lib, name).restype = d
        lib.orc_mu.argtypes = [d, d, d, d]
        lib.orc_p0.argtypes = [d, d, d]
        lib.orc_ptilde.argtypes = [d, d, d, d, d]
        lib.orc_omega_rho.argtypes = [P, d]
        lib.orc_omega_rho.restype = d
        lib.orc_omega_phi.argtypes = [P]
        lib.orc_omega_phi.restype = d
        lib.orc_init.argtypes = [P, _D, _D, _D, _D, _D, _D]
        lib.orc_step.argtypes = [P, _D, _D, _D, _D]
        lib.orc_run.argtypes = [P, _D, _D, ctypes.c_long]
        lib.orc_fields.argtypes = [P, _D, _D, _D, _D, _D, _D, _D]
        _lib = lib
    return _lib


def _cp(p: Params) -> _CParams:
    return _CParams(**{f.name: getattr(p, f.name) for f in fields(Params)})


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _plane(p: Params, a, name):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (p.ny, p.nx):
        raise ValueError(f"{name} must have shape (ny, nx) = {(p.ny, p.nx)}, got {a.shape}")
    return a


def _pops(p: Params, a, name):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (9, p.ny, p.nx):
        raise ValueError(f"{name} must have shape (9, ny, nx), got {a.shape}")
    return a


def check(p: Params) -> int:
    return _load().orc_check(ctypes.byref(_cp(p)))


def stencil(p: Params, phi):
    """Gradient and Laplacian of a phi plane (Eq. (12)) -> (dx, dy, lap)."""
    phi = _plane(p, phi, "phi")
    out = [np.empty_like(phi) for _ in range(3)]
    _load().orc_stencil(ctypes.byref(_cp(p)), _ptr(phi), *(_ptr(o) for o in out))
    return tuple(out)


def feq(rho, ux, uy, pt, gamma, dpx, dpy):
    out = np.empty(9)
    _load().orc_feq(rho, ux, uy, pt, gamma, dpx, dpy, _ptr(out))
    return out


def geq(phi, mu, ux, uy, Gamma):
    out = np.empty(9)
    _load().orc_geq(phi, mu, ux, uy, Gamma, _ptr(out))
    return out


def tmatrix(ux, uy):
    out = np.empty(81)
    _load().orc_tmatrix(ux, uy, _ptr(out))
    return out.reshape(9, 9)


def keq(rho, ux, uy, pt, gamma, dpx, dpy, lap, k8_printed=0):
    out = np.empty(9)
    _load().orc_keq(rho, ux, uy, pt, gamma, dpx, dpy, lap, int(k8_printed), _ptr(out))
    return out


def guo(ux, uy, Fx, Fy):
    out = np.empty(9)
    _load().orc_guo(ux, uy, Fx, Fy, _ptr(out))
    return out


def mu(a, gamma, phi, lap):
    return _load().orc_mu(a, gamma, phi, lap)


def p0(a, rho, phi):
    return _load().orc_p0(a, rho, phi)


def ptilde(a, gamma, rho, phi, lap):
    return _load().orc_ptilde(a, gamma, rho, phi, lap)


def omega_rho(p: Params, phi):
    return _load().orc_omega_rho(ctypes.byref(_cp(p)), phi)


def omega_phi(p: Params):
    return _load().orc_omega_phi(ctypes.byref(_cp(p)))


def collide_f(p: Params, f9, phi, dpx, dpy, lap):
    """Post-collision f at one node -> (fstar[9], (ux, uy))."""
    f9 = np.ascontiguousarray(f9, dtype=np.float64)
    out = np.empty(9)
    u = np.empty(2)
    _load().orc_collide_f(ctypes.byref(_cp(p)), _ptr(f9), phi, dpx, dpy, lap, _ptr(out), _ptr(u))
    return out, (u[0], u[1])


def collide_g(p: Params, g9, phi, lap, ux, uy):
    g9 = np.ascontiguousarray(g9, dtype=np.float64)
    out = np.empty(9)
    _load().orc_collide_g(ctypes.byref(_cp(p)), _ptr(g9), phi, lap, ux, uy, _ptr(out))
    return out


def init(p: Params, phi0, rho0=None, ux0=None, uy0=None):
    """Equilibrium populations of (phi0, rho0, u0) -> (f, g), each (9, ny, nx)."""
    phi0 = _plane(p, phi0, "phi0")
    rho0, ux0, uy0 = (_plane(p, v, n) for v, n in ((rho0, "rho0"), (ux0, "ux0"), (uy0, "uy0")))
    f = np.empty((9, p.ny, p.nx))
    g = np.empty((9, p.ny, p.nx))
    rc = _load().orc_init(ctypes.byref(_cp(p)), _ptr(phi0), _ptr(rho0), _ptr(ux0), _ptr(uy0),
                          _ptr(f), _ptr(g))
    if rc:
        raise ValueError(f"orc_init failed ({rc})")
    return f, g


def step(p: Params, f, g):
    """One time step; returns new (f, g) arrays, inputs untouched."""
    f = _pops(p, f, "f")
    g = _pops(p, g, "g")
    fo = np.empty_like(f)
    go = np.empty_like(g)
    rc = _load().orc_step(ctypes.byref(_cp(p)), _ptr(f), _ptr(g), _ptr(fo), _ptr(go))
    if rc:
        raise ValueError(f"orc_step failed ({rc})")
    return fo, go


def run(p: Params, f, g, nsteps: int, inplace: bool = False):
    """nsteps steps; returns new (f, g) arrays, inputs untouched (inplace: f and g, C-contiguous
    float64 arrays of shape (9, ny, nx), are advanced in place and returned)."""
    if inplace:
        if not (f.dtype == np.float64 and g.dtype == np.float64 and f.flags.c_contiguous and g.flags.c_contiguous):
            raise ValueError("inplace needs C-contiguous float64 arrays")
        f, g = _pops(p, f, "f"), _pops(p, g, "g")
    else:
        f = _pops(p, f, "f").copy()
        g = _pops(p, g, "g").copy()
    rc = _load().orc_run(ctypes.byref(_cp(p)), _ptr(f), _ptr(g), int(nsteps))
    if rc:
        raise ValueError(f"orc_run failed ({rc})")
    return f, g


def macro(p: Params, f, g):
    """Macroscopic fields -> dict(phi, rho, ux, uy, p0), each (ny, nx)."""
    f = _pops(p, f, "f")
    g = _pops(p, g, "g")
    out = {k: np.empty((p.ny, p.nx)) for k in ("phi", "rho", "ux", "uy", "p0")}
    rc = _load().orc_fields(ctypes.byref(_cp(p)), _ptr(f), _ptr(g), *(_ptr(out[k]) for k in
                            ("phi", "rho", "ux", "uy", "p0")))
    if rc:
        raise ValueError(f"orc_fields failed ({rc})")
    return out
