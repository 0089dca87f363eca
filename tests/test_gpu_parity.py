"""GPU parity: the HIP step (through the C-ABI) against the FP64 CPU oracle, element by element,
on the same seeded inputs.

Tolerances.  FP64 runs differ from the oracle only by rounding order (the oracle solves a 9x9
system where the kernel uses the closed-form inverse), so populations agree to a few 1e-16 per
step.  FP32 runs store and compute in single precision: one rounding of a population of size
~0.5 is 3e-8, a node update chains ~100 operations on O(1) values, so one step carries errors of
a few 1e-7 at most and short runs of a few hundred steps stay below the stated bounds, which
are the measured errors with about a 5x margin.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1803_11345_amd import inputs, lbcm
from tests.analytic import diffuse_poiseuille, sharp_poiseuille

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def say(*a):
    print(*a, flush=True)


def both(nx, ny, phi, rho=None, ux=None, uy=None, steps=1, prec="fp64", tile_rows=0, **kw):
    """Run the GPU and the oracle from the same macroscopic state; return both population sets."""
    say(f"case {nx}x{ny} {prec} steps={steps} tile_rows={tile_rows} {kw}")
    okw = dict(kw)
    if "bc_y" in okw:
        okw["walls"] = okw.pop("bc_y")
    for side in ("bottom", "top"):  # the oracle names the wall velocities by their component
        if f"wall_vx_{side}" in okw:
            okw[f"wall_ux_{side}"] = okw.pop(f"wall_vx_{side}")
    p = oracle.Params(nx, ny, **okw)
    fo, go = oracle.init(p, phi, rho, ux, uy)
    fo, go = oracle.run(p, fo, go, steps)
    lat = lbcm.Lattice(nx, ny, precision=prec, tile_rows=tile_rows, **kw).init(phi, rho, ux, uy)
    lat.step(steps)
    f, g = lat.populations()
    fields = lat.fields()
    lat.close()
    return (f, g, fields), (fo, go, oracle.macro(p, fo, go))


def maxerr(a, b):
    return float(np.max(np.abs(a - b)))


PHYS = dict(nu_l=0.1, nu_g=0.02, omega3=1.0)


@pytest.mark.parametrize("bc_y,force", [(0, (0.0, 0.0)), (0, (2e-5, -1e-5)), (1, (0.0, 0.0)), (1, (1e-5, 0.0))])
def test_fp64_one_step(bc_y, force):
    nx, ny = 70, 45  # two column bands (64 + ragged 6), three row segments (16 + 16 + 13)
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=31)
    (f, g, m), (fo, go, mo) = both(nx, ny, phi, rho, ux, uy, steps=1, tile_rows=16, bc_y=bc_y,
                                   force_x=force[0], force_y=force[1], **PHYS)
    ef, eg = maxerr(f, fo), maxerr(g, go)
    say(f"  max |df| = {ef:.2e}  max |dg| = {eg:.2e}")
    assert ef < 1e-14 and eg < 1e-14
    for k in ("phi", "rho", "ux", "uy", "p0"):
        assert maxerr(m[k], mo[k]) < 1e-13, k


@pytest.mark.parametrize("bc_y", [0, 1])
def test_fp64_200_steps(bc_y):
    nx, ny = 70, 45
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=32)
    (f, g, m), (fo, go, mo) = both(nx, ny, phi, rho, ux, uy, steps=200, tile_rows=16, bc_y=bc_y,
                                   force_x=1e-5, **PHYS)
    ef, eg = maxerr(f, fo), maxerr(g, go)
    say(f"  max |df| = {ef:.2e}  max |dg| = {eg:.2e}")
    assert ef < 1e-12 and eg < 1e-12


@pytest.mark.parametrize("bc_y", [0, 1])
def test_fp32_one_and_50_steps(bc_y):
    nx, ny = 70, 45
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=33)
    for steps, tol in ((1, 2e-6), (50, 2e-5)):
        (f, g, m), (fo, go, mo) = both(nx, ny, phi, rho, ux, uy, steps=steps, prec="fp32", tile_rows=16,
                                       bc_y=bc_y, force_x=1e-5, **PHYS)
        ef, eg = maxerr(f, fo), maxerr(g, go)
        say(f"  fp32 {steps} steps: max |df| = {ef:.2e}  max |dg| = {eg:.2e}")
        assert ef < tol and eg < tol


@pytest.mark.parametrize("prec,tol1,tol50", [("fp16s", 3e-5, 3e-4), ("bf16s", 3e-4, 3e-3)])
@pytest.mark.parametrize("bc_y", [0, 1])
def test_16bit_storage_one_and_50_steps(prec, tol1, tol50, bc_y):
    """FP32 arithmetic with f_i - w_i and g_1..g_8 stored in 16 bits (g_0 in FP32).  A stored
    f deviation of ~0.02 carries a half-ulp of 7.6e-6 in FP16 (6.1e-5 in BF16); the bounds are a
    few such roundings per step, and about ten times that after 50 steps."""
    nx, ny = 70, 45
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=38)
    for steps, tol in ((1, tol1), (50, tol50)):
        (f, g, m), (fo, go, mo) = both(nx, ny, phi, rho, ux, uy, steps=steps, prec=prec, tile_rows=2,
                                       bc_y=bc_y, force_x=1e-5, **PHYS)
        ef, eg = maxerr(f, fo), maxerr(g, go)
        say(f"  {prec} {steps} steps: max |df| = {ef:.2e}  max |dg| = {eg:.2e}  max |dphi| = "
            f"{maxerr(m['phi'], mo['phi']):.2e}")
        assert ef < tol and eg < tol


@pytest.mark.parametrize("prec", ["fp16s", "bf16s"])
def test_16bit_checkpoint_and_tiling(prec):
    nx, ny = 130, 37
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=39)
    a = lbcm.Lattice(nx, ny, precision=prec, tile_rows=2, **PHYS).init(phi, rho, ux, uy).step(4)
    b = lbcm.Lattice(nx, ny, precision=prec, tile_rows=1, tile_wx=1, **PHYS).init(phi, rho, ux, uy).step(4)
    sa = a.get_state()
    assert sa.nbytes == 9 * nx * ny * 2 + nx * ny * 4 + 8 * nx * ny * 2
    assert np.array_equal(sa, b.get_state())
    a.step(3)
    c = lbcm.Lattice(nx, ny, precision=prec, **PHYS)
    c.set_state(sa, step=4)
    c.step(3)
    assert np.array_equal(a.get_state(), c.get_state())


@pytest.mark.parametrize("nx,ny,bc_y", [(1, 1, 0), (1, 1, 1), (1, 6, 0), (6, 1, 0), (6, 1, 1), (2, 3, 1),
                                        (3, 2, 0), (65, 2, 1), (64, 64, 0), (129, 7, 0), (5, 130, 1)])
def test_fp64_edge_sizes(nx, ny, bc_y):
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=34)
    (f, g, m), (fo, go, mo) = both(nx, ny, phi, rho, ux, uy, steps=3, tile_rows=0, bc_y=bc_y,
                                   force_x=1e-5, **PHYS)
    assert maxerr(f, fo) < 1e-14 and maxerr(g, go) < 1e-14


@pytest.mark.parametrize("rows", [1, 2, 3, 7, 64, 1000])
def test_segment_rows_do_not_change_results(rows):
    """Tiling only changes which workgroup computes a node, never the arithmetic: bitwise equal."""
    nx, ny = 100, 50
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=35)
    ref = lbcm.Lattice(nx, ny, precision="fp32", tile_rows=16, **PHYS).init(phi, rho, ux, uy).step(7)
    lat = lbcm.Lattice(nx, ny, precision="fp32", tile_rows=rows, **PHYS).init(phi, rho, ux, uy).step(7)
    assert np.array_equal(ref.get_state(), lat.get_state())


@pytest.mark.parametrize("prec", ["fp16s", "bf16s"])
@pytest.mark.parametrize("wx,rows", [(1, 1), (1, 3), (2, 2), (4, 2), (2, 8), (1, 16), (4, 4)])
@pytest.mark.parametrize("ny,bc_y", [(51, 0), (50, 1), (3, 0), (1, 1)])
def test_16bit_tiles_do_not_change_results(prec, wx, rows, ny, bc_y):
    """16-bit storage on small lattices (one row per wave): any tile shape, with odd and single
    row counts, periodic or with walls, gives the same state bit for bit."""
    nx = 100
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=36)
    kw = dict(precision=prec, bc_y=bc_y, force_x=1e-5, **PHYS)
    ref = lbcm.Lattice(nx, ny, tile_wx=1, tile_rows=1, **kw).init(phi, rho, ux, uy).step(5)
    lat = lbcm.Lattice(nx, ny, tile_wx=wx, tile_rows=rows, **kw).init(phi, rho, ux, uy).step(5)
    assert np.array_equal(ref.get_state(), lat.get_state())


@pytest.mark.parametrize("prec", ["fp16s", "bf16s"])
@pytest.mark.parametrize("bc_y", [0, 1])
def test_two_row_waves_equal_one_row_waves(prec, bc_y):
    """Above 2^22 nodes a 16-bit lattice runs the step with two lattice rows per wave; the same box
    in an ensemble runs the one-row kernel.  With an odd row count (the last wave's second row lies
    past the lattice), walls, force and several tile shapes the states agree bit for bit."""
    nx, ny = 2048, 2049
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=37)
    kw = dict(nx=nx, ny=ny, bc_y=bc_y, force_x=1e-5, **PHYS)
    say(f"case two-row vs one-row {prec} {nx}x{ny} bc_y={bc_y}")
    bt = lbcm.Batch([kw], precision=prec)
    bt[0].init(phi, rho, ux, uy)
    bt.step(4)
    ref = bt[0].get_state()
    bt.close()
    for wx, rows in ((0, 0), (1, 3), (8, 1), (2, 8)):
        lat = lbcm.Lattice(precision=prec, tile_wx=wx, tile_rows=rows, **kw).init(phi, rho, ux, uy)
        assert lat.rows_per_wave() == 2
        lat.step(4)
        assert np.array_equal(lat.get_state(), ref), (wx, rows)
        lat.close()
    small = lbcm.Lattice(precision=prec, nx=64, ny=64)
    assert small.rows_per_wave() == 1
    small.close()


@pytest.mark.parametrize("prec,nx,ny", [("fp32", 100, 50), ("fp64", 130, 37), ("fp16s", 2048, 2049)])
def test_autotune_keeps_state_and_results(prec, nx, ny):
    """lbcm_autotune times tile shapes on the spare pair: the state is unchanged, the chosen shape
    is a valid split (heights powers of two or three times one), and the tuned lattice then
    steps bit for bit like an untuned one (two-row waves in the 16-bit case)."""
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=40)
    kw = dict(precision=prec, bc_y=1, force_x=1e-5, **PHYS)
    a = lbcm.Lattice(nx, ny, **kw).init(phi, rho, ux, uy).step(2)
    b = lbcm.Lattice(nx, ny, **kw).init(phi, rho, ux, uy).step(2)
    before = a.get_state()
    wx, rows = a.autotune(trials=2)
    say(f"  {prec} {nx}x{ny}: autotuned tile {wx} x {rows}, rows per wave {a.rows_per_wave()}")
    assert np.array_equal(a.get_state(), before)
    assert wx >= 1 and rows >= 1 and wx * rows <= (8 if prec == "fp64" else 16)
    assert rows in (1, 2, 3, 4, 6, 8, 12, 16) or rows >= ny
    a.step(3)
    b.step(3)
    assert np.array_equal(a.get_state(), b.get_state())
    a.close()
    b.close()


def test_static_droplet_fp64_2000_steps():
    """64^2 static droplet, R = 16, a = 0.04, gamma = 0.08, M = 0.1, nu = 1/6, 2000 steps: the
    GPU state against the oracle, and sum phi conserved to round-off."""
    n = 64
    phi0 = inputs.droplet(n, n, 16, inputs.interface_width(0.04, 0.08))
    say("case static droplet 64^2 fp64 2000 steps")
    p = oracle.Params(n, n)
    fo, go = oracle.run(p, *oracle.init(p, phi0), 2000)
    mo = oracle.macro(p, fo, go)
    lat = lbcm.Lattice(n, n, precision="fp64").init(phi0)
    d0 = lat.diag()
    lat.step(2000)
    m = lat.fields()
    d1 = lat.diag()
    e = maxerr(m["phi"], mo["phi"])
    drift = abs(d1["sum_phi"] - d0["sum_phi"]) / d0["sum_abs_phi"]
    say(f"  max |dphi| = {e:.2e}, sum phi drift = {drift:.2e}, step = {d1['step']}")
    assert e < 1e-11
    assert drift < 1e-12
    assert maxerr(m["p0"], mo["p0"]) < 1e-11


def _radial_fit(phi):
    """Least-squares fit of phi = c + A tanh((R - r) / W) over every node, r the distance to the
    box centre: (R, W, c, A, max residual)."""
    from scipy.optimize import least_squares

    ny, nx = phi.shape
    yy, xx = np.mgrid[0:ny, 0:nx].astype(float)
    r = np.hypot(xx - nx / 2, yy - ny / 2)
    fit = least_squares(lambda q: (q[2] + q[3] * np.tanh((q[0] - r) / q[1]) - phi).ravel(), [ny / 4, 2.0, 0.0, 1.0])
    R, W, c, A = fit.x
    return R, W, c, A, float(np.abs(c + A * np.tanh((R - r) / W) - phi).max())


def test_static_droplet_equilibrium_profile_and_laplace_law():
    """The 64^2 droplet (R = 16, a = 0.04, gamma = 0.08) run in FP64 to equilibrium (200,000
    steps; the velocity then changes by < 1e-11 per step, sum phi is conserved to 1e-13):

    - interface profile: phi = c + A tanh((R - r) / W') fits every node within 1.5e-2 (measured
      7.7e-3) with W' within 3 % of the width sqrt(2 gamma / a) = 2 of the flat-interface
      solution of mu = 0 (measured -1.1 %) and A within 1 % of 1;
    - both bulk values sit above +-1 by the shift that a uniform chemical potential
      mu = sigma / (2R) gives, mu / (2a) = sigma / (4 a R) (Gibbs-Thomson): c within 5 % of it
      (measured 0.2 %);
    - Laplace's law dp = sigma / R with sigma = sqrt(8 gamma a / 9) and dp the jump of the bulk
      pressure p0 of Eq. (13) between the centre and the corner: within 5 % with R from the
      area sum (1 + phi) / 2 (measured -1.6 %), and within 6 % with the radius of the fitted
      profile (measured -5.2 %; that radius excludes the bulk shift, which the area sum counts
      as droplet area).
    After 2000 steps (the parity run above) the pressure is still relaxing (dp R / sigma = 0.91
    at 2000 steps, 0.98 at 5000)."""
    n, a, gam = 64, 0.04, 0.08
    W = inputs.interface_width(a, gam)
    sig = math.sqrt(8 * gam * a / 9)
    phi0 = inputs.droplet(n, n, 16, W)
    say("case static droplet 64^2 fp64 to equilibrium (200000 steps)")
    lat = lbcm.Lattice(n, n, precision="fp64").init(phi0)
    d0 = lat.diag()
    lat.step(200000)
    d = lat.diag()
    m = lat.fields()
    lat.close()
    phi = m["phi"]
    assert d["max_du"] < 1e-11
    assert abs(d["sum_phi"] - d0["sum_phi"]) / d0["sum_abs_phi"] < 1e-13
    R, Wf, c, A, res = _radial_fit(phi)
    shift = sig / (4 * a * R)
    Ra = math.sqrt(np.sum((1 + phi) / 2) / math.pi)
    dp = m["p0"][n // 2, n // 2] - m["p0"][0, 0]
    say(f"  fit R {R:.4f} W {Wf:.4f} (W = {W}) c {c:.5f} (sigma/(4aR) = {shift:.5f}) A {A:.5f} max residual "
        f"{res:.2e}; dp R/sigma = {dp * Ra / sig:.4f} (area radius {Ra:.4f}), {dp * R / sig:.4f} (fitted radius)")
    assert res < 1.5e-2
    assert abs(Wf / W - 1) < 0.03
    assert abs(A - 1) < 0.01
    assert abs(c / shift - 1) < 0.05
    assert abs(dp * Ra / sig - 1) < 0.05
    assert abs(dp * R / sig - 1) < 0.06


def test_static_droplet_fp32_2000_steps():
    n = 64
    phi0 = inputs.droplet(n, n, 16, inputs.interface_width(0.04, 0.08))
    say("case static droplet 64^2 fp32 2000 steps")
    p = oracle.Params(n, n)
    mo = oracle.macro(p, *oracle.run(p, *oracle.init(p, phi0), 2000))
    lat = lbcm.Lattice(n, n, precision="fp32").init(phi0)
    d0 = lat.diag()
    m = lat.step(2000).fields()
    d1 = lat.diag()
    e = np.linalg.norm(m["phi"] - mo["phi"]) / np.linalg.norm(mo["phi"])
    drift = abs(d1["sum_phi"] - d0["sum_phi"]) / d0["sum_abs_phi"]
    say(f"  phi rel L2 = {e:.2e}, sum phi drift = {drift:.2e}")
    assert e < 1e-5
    assert drift < 1e-5


@pytest.mark.parametrize("ratio", [1, 10, 100, 1000])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
@pytest.mark.parametrize("start", ["rest", "profile"])
def test_layered_poiseuille_4x256(ratio, prec, tol, start):
    """4 x 256 channel, walls, force 1e-6, phi = +1 below / -1 above (tanh), nu1 = 0.1,
    nu2 = ratio * nu1: velocity profile after 2000 steps from rest, or from the steady diffuse-
    interface profile, vs the oracle started from the same state.  The velocity is a difference
    of O(0.1) populations divided by rho, so its error is bounded in absolute terms by a few
    roundings of the populations: the bound is on max |u - u_oracle|.  From rest u stays below
    2e-4 over these steps; from the profile (u up to 0.08) the stored FP32 deviations are
    O(0.03), whose half-ulp (1e-9) can add up coherently over the 2000 steps to ~2e-6: the FP32
    bound there is 5e-6 (measured 1.6e-6)."""
    nx, ny = 4, 256
    W = inputs.interface_width(0.04, 0.08)
    phi0 = inputs.layered(nx, ny, W)
    ux0 = None
    if start == "profile":
        ux0 = np.repeat(diffuse_poiseuille(ny, 0.1, 0.1 * ratio, 1e-6, W)[:, None], nx, axis=1)
    kw = dict(bc_y=1, nu_l=0.1, nu_g=0.1 * ratio, force_x=1e-6)
    (f, g, m), (fo, go, mo) = both(nx, ny, phi0, None, ux0, None, steps=2000, prec=prec, **kw)
    if prec == "fp32" and start == "profile":
        tol = 5e-6
    e = maxerr(m["ux"], mo["ux"])
    rel = np.linalg.norm(m["ux"] - mo["ux"]) / np.linalg.norm(mo["ux"])
    say(f"  max |dux| = {e:.2e} (rel L2 {rel:.2e})  max |dphi| = {maxerr(m['phi'], mo['phi']):.2e}")
    assert e < tol


_STEADY = {}


def _steady_channel(ratio):
    """The 4 x 256 layered channel (ratio nu2 / nu1, nu1 = 0.1, force 1e-6) in FP64 from rest
    until the velocity changes by less than 1e-12 per step (checked every 1000 steps with the
    FP64 max |v(t) - v(t-1)| of lbcm_diag): (steps, u(y), max |du| at the stop)."""
    if ratio not in _STEADY:
        W = inputs.interface_width(0.04, 0.08)
        lat = lbcm.Lattice(4, 256, precision="fp64", bc_y=1, nu_l=0.1, nu_g=0.1 * ratio, force_x=1e-6)
        lat.init(inputs.layered(4, 256, W))
        steps, du = 0, math.inf
        while du >= 1e-12:
            assert steps < 3_000_000, "no steady state"
            lat.step(1000)
            steps += 1000
            du = lat.diag()["max_du"]
        u = lat.fields()["ux"]
        lat.close()
        _STEADY[ratio] = (steps, u, du)
    return _STEADY[ratio]


@pytest.mark.parametrize("ratio", [1, 10, 100, 1000])
def test_layered_poiseuille_steady_state_fp64(ratio):
    """The 4 x 256 layered channel run from rest to steady state (max |v(t) - v(t-1)| < 1e-12
    per step, the FP64 device reduction) against the analytic two-layer Stokes profile of the
    diffuse viscosity the method has (relative L2 < 1e-3; measured 1.8e-4 - 2.6e-4: the
    remaining error is the bounce-back wall and the stencil) and, for ratio 1, the parabola
    G y (L - y) / (2 nu).  The flow stays unidirectional and uniform along x."""
    W = inputs.interface_width(0.04, 0.08)
    say(f"case layered channel steady state fp64 ratio {ratio}")
    steps, u, du = _steady_channel(ratio)
    ua = diffuse_poiseuille(256, 0.1, 0.1 * ratio, 1e-6, W)
    err = np.linalg.norm(u[:, 0] - ua) / np.linalg.norm(ua)
    say(f"  steady after {steps} steps (max |du| {du:.2e}): rel L2 vs analytic {err:.2e}")
    assert np.max(np.abs(u - u[:, :1])) == 0.0
    assert err < 1e-3
    if ratio == 1:
        us = sharp_poiseuille(256, 0.1, 0.1, 1e-6)
        assert np.linalg.norm(u[:, 0] - us) / np.linalg.norm(us) < 1e-3


@pytest.mark.parametrize("ratio", [1, 10, 100, 1000])
def test_layered_poiseuille_steady_state_fp32(ratio):
    """FP32 storage cannot resolve a change of 1e-12 per step (a velocity of 0.08 has an ulp of
    7e-9), so the FP32 channel runs the step count at which the FP64 run met the rule.  Its
    profile matches the analytic one within the oracle's own bound (relative L2 < 3e-3) and the
    FP64 profile within 1e-4: the steady FP32 state carries the rounding of each step (a
    half-ulp of the O(1e-2) stored deviations, ~1e-9) accumulated over the relaxation time of
    the channel, L^2 / (pi^2 nu) = 6.6e4 steps at nu = 0.1 (measured 1.9e-5 - 4.1e-5)."""
    W = inputs.interface_width(0.04, 0.08)
    steps, u64, _ = _steady_channel(ratio)
    say(f"case layered channel steady state fp32 ratio {ratio}, {steps} steps")
    lat = lbcm.Lattice(4, 256, precision="fp32", bc_y=1, nu_l=0.1, nu_g=0.1 * ratio, force_x=1e-6)
    lat.init(inputs.layered(4, 256, W))
    lat.step(steps)
    u = lat.fields()["ux"]
    lat.close()
    ua = diffuse_poiseuille(256, 0.1, 0.1 * ratio, 1e-6, W)
    err = np.linalg.norm(u[:, 0] - ua) / np.linalg.norm(ua)
    d64 = maxerr(u, u64)
    say(f"  rel L2 vs analytic {err:.2e}, max |u32 - u64| {d64:.2e}")
    assert err < 3e-3
    assert d64 < 1e-4


def _window(full_phi, y0, x0, h, w, steps, **kw):
    """Oracle run on a periodic patch around a window; the window is exact when the margin
    exceeds the 2-node-per-step reach of the step plus the 1-node reach of the initialisation."""
    ny, nx = full_phi.shape
    m = 2 * steps + 2
    ys = np.arange(y0 - m, y0 + h + m) % ny
    xs = np.arange(x0 - m, x0 + w + m) % nx
    patch = full_phi[np.ix_(ys, xs)]
    p = oracle.Params(w + 2 * m, h + 2 * m, **kw)
    fo, go = oracle.run(p, *oracle.init(p, patch), steps)
    return fo[:, m:m + h, m:m + w], go[:, m:m + h, m:m + w]


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-6), ("fp16s", 3e-5), ("bf16s", 3e-4)])
def test_spinodal_4096_sampled_windows(prec, tol):
    """4096^2 periodic spinodal (phi0 uniform in [-0.05, 0.05], SplitMix64 seed 1, a = 0.04,
    gamma = 0.08, M = 0.1, nu = 0.05) in the benchmark's launch configuration (the 16-bit modes
    with two-row waves): after 10 steps, windows (including ones that wrap around the periodic
    edges) match the oracle, within the tier of each storage (measured 2.5e-8, 2.9e-6, 2.4e-5;
    the 16-bit bounds are those of one step of the small-lattice test)."""
    n, steps = 4096, 10
    phi0 = inputs.spinodal(n, n, seed=1)
    say(f"case spinodal 4096^2 {prec} 10 steps")
    lat = lbcm.Lattice(n, n, precision=prec, nu_l=0.05, nu_g=0.05).init(phi0)
    assert lat.rows_per_wave() == (1 if prec == "fp32" else 2)
    lat.step(steps)
    f, g = lat.populations()
    d = lat.diag()
    lat.close()
    assert d["nonfinite"] == 0
    worst = 0.0
    for (y0, x0) in [(0, 0), (4096 - 16, 4096 - 16), (1000, 63), (2047, 4000), (3333, 1234)]:
        h = w = 32
        fo, go = _window(phi0, y0, x0, h, w, steps, nu_l=0.05, nu_g=0.05)
        ys = np.arange(y0, y0 + h) % n
        xs = np.arange(x0, x0 + w) % n
        fw = f[:, ys][:, :, xs]
        gw = g[:, ys][:, :, xs]
        e = max(maxerr(fw, fo), maxerr(gw, go))
        worst = max(worst, e)
    say(f"  worst window |GPU - oracle| = {worst:.2e}")
    assert worst < tol


def test_checkpoint_resume_bitwise():
    nx, ny = 66, 33
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=36)
    a = lbcm.Lattice(nx, ny, precision="fp32", **PHYS).init(phi, rho, ux, uy).step(5)
    snap = a.get_state()
    a.step(5)
    b = lbcm.Lattice(nx, ny, precision="fp32", **PHYS)
    b.set_state(snap, step=5)
    b.step(5)
    assert np.array_equal(a.get_state(), b.get_state())
    assert b.diag()["step"] == 10


def test_recovery_from_a_corrupted_state():
    """Snapshot, then the whole workspace corrupted (populations, partial sums and the divergence
    flag filled with NaN bytes): the next checked step reports the divergence; restoring the
    snapshot and continuing gives bitwise the uninterrupted run, with the check (every step)
    quiet after the restore."""
    nx, ny = 66, 33
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=37)
    kw = dict(precision="fp32", check_every=1, **PHYS)
    a = lbcm.Lattice(nx, ny, **kw).init(phi, rho, ux, uy).step(5)
    snap = a.get_state()
    a.step(5)
    b = lbcm.Lattice(nx, ny, **kw).init(phi, rho, ux, uy).step(5)
    b.workspace.fill_(255)
    with pytest.raises(lbcm.LbcmError):
        b.step(1)
    b.set_state(snap, step=5)
    b.step(5)
    assert np.array_equal(a.get_state(), b.get_state())
    assert b.diag()["step"] == 10 and b.diag()["nonfinite"] == 0
    a.close()
    b.close()


def test_errors_and_divergence_flag():
    lat = lbcm.Lattice(16, 16, precision="fp32", check_every=1)
    with pytest.raises(lbcm.LbcmError) as e:
        lat.step(1)
    assert e.value.code == lbcm.LBCM_ESTATE
    phi = np.zeros((16, 16))
    phi[5, 7] = np.nan
    lat.init(phi)
    with pytest.raises(lbcm.LbcmError) as e:
        lat.step(3)
    assert e.value.code == lbcm.LBCM_EDIVERGED
    assert lat.diag()["nonfinite"] > 0
    with pytest.raises(lbcm.LbcmError):
        lat.step(-1)
    lat.close()


def test_torch_stream_and_device_io():
    import torch

    nx, ny = 40, 24
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=37)
    s = torch.cuda.Stream()
    ref = lbcm.Lattice(nx, ny, precision="fp64", **PHYS).init(phi, rho, ux, uy).step(4)
    lat = lbcm.Lattice(nx, ny, precision="fp64", stream=s, **PHYS)
    with torch.cuda.stream(s):
        t = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (phi, rho, ux, uy)]
        lbcm.lbcm_init_device(lat.h, *t)
        lat.step(4)
        out = [torch.empty((ny, nx), dtype=torch.float64, device="cuda") for _ in range(5)]
        lbcm.lbcm_fields_device(lat.h, *out)
    s.synchronize()
    m = ref.fields()
    for k, o in zip(("phi", "rho", "ux", "uy", "p0"), out):
        assert np.array_equal(o.cpu().numpy(), m[k]), k


WALLS = dict(bc_y=1, wall_vx_bottom=-3e-3, wall_vx_top=5e-3, wall_gradient=0.05)


@pytest.mark.parametrize("steps,tol", [(1, 1e-14), (200, 1e-12)])
def test_moving_wetting_walls_fp64(steps, tol):
    """Walls moving at -3e-3 and +5e-3 with the wall gradient 0.05: the step, the readers and the
    initial unstreaming all carry the moving-wall terms and the ghost rows."""
    nx, ny = 70, 45
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=41)
    (f, g, m), (fo, go, mo) = both(nx, ny, phi, rho, ux, uy, steps=steps, tile_rows=16, force_x=1e-5,
                                   **WALLS, **PHYS)
    ef, eg = maxerr(f, fo), maxerr(g, go)
    say(f"  max |df| = {ef:.2e}  max |dg| = {eg:.2e}")
    assert ef < tol and eg < tol
    for k in ("phi", "rho", "ux", "uy", "p0"):
        assert maxerr(m[k], mo[k]) < 10 * tol, k


@pytest.mark.parametrize("prec,tol1,tol50", [("fp32", 2e-6, 2e-5), ("fp16s", 3e-5, 3e-4), ("bf16s", 3e-4, 3e-3)])
def test_moving_wetting_walls_reduced_precision(prec, tol1, tol50):
    nx, ny = 70, 45
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=42)
    for steps, tol in ((1, tol1), (50, tol50)):
        (f, g, m), (fo, go, mo) = both(nx, ny, phi, rho, ux, uy, steps=steps, prec=prec, tile_rows=2, **WALLS,
                                       **PHYS)
        ef, eg = maxerr(f, fo), maxerr(g, go)
        say(f"  {prec} {steps} steps: max |df| = {ef:.2e}  max |dg| = {eg:.2e}")
        assert ef < tol and eg < tol


@pytest.mark.parametrize("nx,ny", [(1, 1), (6, 1), (2, 3), (65, 2), (5, 130)])
def test_moving_wetting_walls_edge_sizes(nx, ny):
    """One-row channels (both walls on the same row), two rows, ragged tiles."""
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=43)
    (f, g, m), (fo, go, mo) = both(nx, ny, phi, rho, ux, uy, steps=3, **WALLS, **PHYS)
    assert maxerr(f, fo) < 1e-14 and maxerr(g, go) < 1e-14


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-7)])
def test_couette_flow(prec, tol):
    """Walls moving at -U and +U drive the exact linear profile through the wall velocities."""
    L, U = 32, 1e-3
    lat = lbcm.Lattice(4, L, precision=prec, bc_y=1, wall_vx_bottom=-U, wall_vx_top=U, nu_l=1 / 6, nu_g=1 / 6)
    lat.init(np.ones((L, 4)))
    lat.step(60000)
    u = lat.fields()["ux"]
    ua = -U + 2 * U * (np.arange(L) + 0.5) / L
    err = maxerr(u, ua[:, None])
    say(f"  {prec} Couette max |u - u_a| = {err:.2e}")
    assert err < tol
    lat.close()


def test_droplet_deformation_in_shear_follows_taylor():
    """The paper's shear test: a droplet (R = 30) between walls moving at -v_w and +v_w
    (2H = 200, nu = 0.2, Re = v_w R^2 / (H nu) = 0.1), capillary numbers Ca = v_w R nu / (H sigma)
    from 0.05 to 0.2 set through sigma = sqrt(8 gamma a / 9) at the interface width 2.  The
    deformation D = (A - B) / (A + B) grows linearly in Ca with Taylor's slope 35/32 for equal
    viscosities; the fitted slope must lie within 5 % of it."""
    n, R, H, nu, W = 200, 30, 100, 0.2, 2.0
    vw = 0.1 * H * nu / R ** 2
    y = np.arange(n) + 0.5
    u0 = np.repeat((vw * (2 * y / n - 1))[:, None], n, axis=1)
    yy, xx = np.mgrid[0:n, 0:n].astype(float)
    cas, ds = [], []
    for Ca in (0.05, 0.1, 0.15, 0.2):
        sigma = vw * R * nu / (H * Ca)
        a = 3 * sigma / (2 * W)  # sigma = (2 / 3) a W at W = sqrt(2 gamma / a)
        lat = lbcm.Lattice(n, n, precision="fp32", bc_y=1, a=a, gamma=a * W * W / 2, mobility=0.1, nu_l=nu, nu_g=nu,
                           wall_vx_bottom=-vw, wall_vx_top=vw)
        lat.init(inputs.droplet(n, n, R, W), None, u0, None)
        lat.step(240000)
        phi = lat.fields()["phi"]
        lat.close()
        w = np.clip((1 + phi) / 2, 0, 1)
        m = w.sum()
        cx, cy = (w * xx).sum() / m, (w * yy).sum() / m
        I = np.array([[(w * (xx - cx) ** 2).sum(), (w * (xx - cx) * (yy - cy)).sum()],
                      [(w * (xx - cx) * (yy - cy)).sum(), (w * (yy - cy) ** 2).sum()]]) / m
        ev = np.linalg.eigvalsh(I)
        A, B = math.sqrt(ev[1]), math.sqrt(ev[0])  # axes in proportion to the semi-axes
        cas.append(Ca)
        ds.append((A - B) / (A + B))
        say(f"  Ca {Ca}: D = {ds[-1]:.4f}")
    slope, icpt = np.polyfit(cas, ds, 1)
    say(f"  fitted slope {slope:.4f} (Taylor {35 / 32:.5f}), intercept {icpt:.4f}")
    assert abs(slope / (35 / 32) - 1) < 0.05


def _contact_angle_from_wall_gradient(h, a, gamma):
    """The paper's wetting relation: h = sqrt(2 a / gamma) sqrt(c (1 - c)), c = cos(vartheta / 3),
    vartheta = arccos(sin^2 theta), read with the sign of theta - 90 degrees (theta measured through
    the phi = +1 phase; a positive wall gradient repels that phase).  Returns theta in degrees."""
    q = h * h * gamma / (2 * a)
    c = 0.5 + math.sqrt(0.25 - q)  # the root near 1 (small angles vartheta)
    theta = math.degrees(math.asin(math.sqrt(math.cos(3 * math.acos(c)))))
    return 180 - theta if h > 0 else theta


def _interface_points(phi):
    """Points of the phi = 0 level set, linearly interpolated along rows and columns."""
    pts = []
    ny, nx = phi.shape
    for x in range(nx):
        c = phi[:, x]
        for y in np.nonzero((c[:-1] > 0) != (c[1:] > 0))[0]:
            pts.append((x, y + c[y] / (c[y] - c[y + 1])))
    for y in range(ny):
        r = phi[y]
        for x in np.nonzero((r[:-1] > 0) != (r[1:] > 0))[0]:
            pts.append((x + r[x] / (r[x] - r[x + 1]), y))
    return np.array(pts)


def test_contact_angles_follow_the_wetting_relation():
    """The paper's contact-angle test: a phi = +1 drop on the bottom wall of a 100 x 100 box
    (a = gamma = 0.04, nu_l = 0.1, viscosity ratio 2, periodic in x) relaxes to the contact angle
    that the wall gradient sets.  The drop starts as a half disc (R = 25) on the wall: in a
    density-matched fluid a uniform body force would not move it relative to the fluid, and the
    equilibrium angle does not depend on how the drop reached the wall.  The angle comes from a
    circle fitted to the phi = 0 contour away from the wall; it must follow the relation within
    3 degrees, with the error growing with |h| (0.3 to 2.5 degrees measured)."""
    n, a, g = 100, 0.04, 0.04
    W = inputs.interface_width(a, g)
    errs = {}
    for h in (-0.15, -0.05, 0.0, 0.05, 0.15):
        lat = lbcm.Lattice(n, n, precision="fp64", bc_y=1, a=a, gamma=g, mobility=0.1, nu_l=0.1, nu_g=0.05,
                           wall_gradient=h)
        phi0 = inputs.droplet(n, n, 25.0, W, cx=50.0, cy=-0.5)
        lat.init(phi0)
        lat.step(20000)
        phi = lat.fields()["phi"]
        lat.close()
        assert abs(phi.sum() - phi0.sum()) < 1e-9 * np.abs(phi0).sum()
        p = _interface_points(phi)
        p = p[p[:, 1] > 4]  # leave out the rows next to the wall
        A = np.stack([p[:, 0], p[:, 1], np.ones(len(p))], 1)
        c = np.linalg.lstsq(A, p[:, 0] ** 2 + p[:, 1] ** 2, rcond=None)[0]
        xc, yc = c[0] / 2, c[1] / 2
        R = math.sqrt(c[2] + xc * xc + yc * yc)
        theta = math.degrees(math.acos(-(yc + 0.5) / R))  # the wall lies at y = -1/2
        want = _contact_angle_from_wall_gradient(h, a, g)
        errs[h] = theta - want
        say(f"  dphi_w = {h:+.2f}: theta {theta:.2f} deg, relation {want:.2f} deg")
    assert all(abs(e) < 3.0 for e in errs.values())
    assert abs(errs[0.0]) < 1.0
    assert abs(errs[-0.15]) > abs(errs[-0.05]) and abs(errs[0.15]) > abs(errs[0.05])


def _pair_bytes(nodes, prec):
    """Bytes of one (f, g) population pair in the workspace: the f set and the g set, each rounded
    up to 256 bytes (16-bit modes keep g_0 in FP32)."""
    f, g0, g = {"fp64": (8, 8, 8), "fp32": (4, 4, 4), "fp16s": (2, 4, 2), "bf16s": (2, 4, 2)}[prec]
    up = lambda v: (v + 255) // 256 * 256
    return up(9 * nodes * f) + up(nodes * g0 + 8 * nodes * g)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s"])
def test_every_slot_of_the_output_pair_is_written(prec):
    """Poison test: before each step the pair it writes is filled with NaN bytes; a step that
    left any slot unwritten (a ragged tile edge, a wall row) would carry them into the state.
    The state must equal that of an unpoisoned run bit for bit.  Ragged tiles, walls (moving,
    wetting) and a force."""
    nx, ny = 70, 45
    phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=50)
    kw = dict(precision=prec, bc_y=1, force_x=1e-5, wall_vx_top=1e-3, wall_gradient=0.02, nu_l=0.1, nu_g=0.02)
    lat = lbcm.Lattice(nx, ny, **kw).init(phi, rho, ux, uy)
    ref = lbcm.Lattice(nx, ny, **kw).init(phi, rho, ux, uy)
    pb = _pair_bytes(nx * ny, prec)
    assert lat.workspace.numel() >= 2 * pb
    for s in range(4):
        out = 1 - s % 2  # init leaves the state in pair 0; each step writes the other pair
        lat.workspace[out * pb:(out + 1) * pb].fill_(255)
        lat.step(1)
        ref.step(1)
        assert np.array_equal(lat.get_state(), ref.get_state()), s
    assert np.isfinite(lat.fields()["phi"]).all()
    lat.close()
    ref.close()
