"""Pin of the FP64 oracle against an exact-rational brute force of the same step
(tests/rational_step.py: Fractions, the paper's order, k^eq from its definition T^T f^eq, the
inverse of T^T by exact elimination).  The parameters and initial planes are dyadic rationals,
exactly representable in binary, so both start from identical values; the oracle then rounds at
every operation and the rational step does not.  On 3x3 and 4x4 periodic lattices and a 4x4
channel with walls (moving, wetting), with a body force, over 1-3 steps, the oracle's
populations must equal the exact ones to within 1e-15 (populations are O(0.5): that is a few
units in the last place).  The rational step starts from its own exact equilibria, the oracle
from those values rounded once to double; the oracle's own initialisation is compared with the
exact equilibria as well.""" 
from fractions import Fraction as Q

import numpy as np
import pytest

from paper_1803_11345_amd import inputs
from tests import rational_step as rs

PHYS = dict(a=Q(3, 64), gamma=Q(5, 64), mobility=Q(1, 8), Gamma=Q(1), nu_l=Q(1, 8), nu_g=Q(1, 32), omega3=Q(3, 4))


def _phi0(nx, ny, seed):
    """Dyadic phi0 in [-1, 1): multiples of 1/64 from the seeded generator."""
    u = inputs.uniform(seed, nx * ny)
    return [[Q(int(np.floor(128 * u[y * nx + x])) - 64, 64) for x in range(nx)] for y in range(ny)]


def _oracle_params(orc, nx, ny, c_kw):
    kw = {k: float(v) for k, v in PHYS.items()}
    kw.update({k: float(v) for k, v in c_kw.items() if k in ("force_x", "force_y", "wall_ux_bottom", "wall_ux_top",
                                                                  "wall_gradient")})
    return orc.Params(nx, ny, walls=int(c_kw.get("walls", 0)), nthreads=1, **kw)


def _rational_params(c_kw):
    return rs.Phys(PHYS["a"], PHYS["gamma"], PHYS["mobility"], PHYS["Gamma"], PHYS["nu_l"], PHYS["nu_g"],
                   PHYS["omega3"], fx=c_kw.get("force_x", Q(0)), fy=c_kw.get("force_y", Q(0)),
                   walls=int(c_kw.get("walls", 0)), u_bottom=c_kw.get("wall_ux_bottom", Q(0)),
                   u_top=c_kw.get("wall_ux_top", Q(0)), wall_gradient=c_kw.get("wall_gradient", Q(0)))


def _to_array(P, nx, ny):
    return np.array([[[float(P[i][y][x]) for x in range(nx)] for y in range(ny)] for i in range(9)])


CASES = [
    ("periodic 3x3", 3, 3, 1, dict()),
    ("periodic 4x4 force", 4, 4, 3, dict(force_x=Q(1, 1024), force_y=Q(-1, 2048))),
    ("periodic 3x3 force", 3, 3, 3, dict(force_x=Q(-3, 4096))),
    ("channel 4x4 walls force", 4, 4, 3, dict(walls=1, force_x=Q(1, 1024))),
    ("channel 3x4 moving wetting walls", 3, 4, 2,
     dict(walls=1, wall_ux_bottom=Q(-1, 256), wall_ux_top=Q(1, 128), wall_gradient=Q(1, 32))),
]


@pytest.mark.parametrize("name,nx,ny,steps,c_kw", CASES, ids=[c[0] for c in CASES])
def test_oracle_equals_exact_rational_step(orc, name, nx, ny, steps, c_kw):
    c = _rational_params(c_kw)
    p = _oracle_params(orc, nx, ny, c_kw)
    phi0 = _phi0(nx, ny, seed=900 + nx * 10 + ny + steps)
    # the initial equilibria: exact vs oracle
    f, g = rs.init(phi0, nx, ny, c)
    fo, go = orc.init(p, np.array([[float(v) for v in row] for row in phi0]))
    assert max(np.abs(_to_array(f, nx, ny) - fo).max(), np.abs(_to_array(g, nx, ny) - go).max()) < 1e-15
    # the steps: the rational run from its exact equilibria, the oracle from the same values
    # rounded once to double (half an ulp, ~3e-17)
    fo, go = _to_array(f, nx, ny), _to_array(g, nx, ny)
    for s in range(1, steps + 1):
        f, g = rs.step(f, g, nx, ny, c)
        fo, go = orc.step(p, fo, go)
        ef = np.abs(_to_array(f, nx, ny) - fo).max()
        eg = np.abs(_to_array(g, nx, ny) - go).max()
        print(f"{name}: step {s}: max |oracle - exact| f {ef:.2e} g {eg:.2e}")
        assert ef < 1e-15 and eg < 1e-15, (s, ef, eg)
    # the state moved: the comparison is not of a fixed point
    assert np.abs(_to_array(f, nx, ny) - orc.init(p, np.array([[float(v) for v in row] for row in phi0]))[0]).max() > 1e-6


def test_rational_step_conserves_exactly():
    """Sum rho and sum phi are invariants of the periodic step and of the walls, and the momentum
    grows by exactly N F per step: in exact arithmetic these hold with equality."""
    nx, ny = 3, 4
    for kw in (dict(force_x=Q(1, 512)), dict(walls=1)):
        c = _rational_params(kw)
        f, g = rs.init(_phi0(nx, ny, seed=950), nx, ny, c)
        tot = lambda P, w=lambda i: 1: sum(w(i) * P[i][y][x] for i in range(9) for y in range(ny) for x in range(nx))
        m0, p0, j0 = tot(f), tot(g), tot(f, lambda i: rs.CX[i])
        f2, g2 = rs.step(f, g, nx, ny, c)
        assert tot(f2) == m0 and tot(g2) == p0
        if not kw.get("walls"):
            assert tot(f2, lambda i: rs.CX[i]) == j0 + nx * ny * kw["force_x"]
