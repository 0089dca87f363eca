"""Exact-rational brute force of one time step of the hybrid central-moments / BGK scheme, a third
implementation used only to pin the FP64 oracle (test infrastructure; it imports neither the
oracle nor the GPU library).

Every quantity is a ``fractions.Fraction``, so the step is computed without rounding.  The code
follows the paper's statement of the method in its order, on a tiny lattice:

1. phi = sum_i g_i at every node (macroscopic variables after Eq. (14)); behind a half-way wall
   the ghost row holds the wall row's phi minus the wall gradient (reading R18);
2. gradient and Laplacian by the stencils of Eq. (12), coefficient i taken at x + c_i;
3. mu = a (-phi + phi^3) - gamma Lap(phi) (the introduction), p0 of Eq. (13), p~ of Eq. (14);
4. rho = sum_i f_i, v = (sum_i f_i c_i + F / 2) / rho (Guo's half force, reading R8);
5. the relaxation rates after Eq. (14): omega_rho interpolated linearly in phi between omega_g
   and omega_l, omega_phi from the mobility;
6. f^eq of Eqs. (8), (10), (11) (with w^yy_4 = +1/3, reading R1), g^eq of Eqs. (9)-(10);
7. the basis of Eq. (15) evaluated at c - v, k = T^T f, and k^eq = T^T f^eq by its definition
   (not the printed closed forms; reading R2 is what that definition gives), the forcing moments
   R = T^T F^Guo, relaxation Eq. (17) with rates (1, 1, 1, omega3, omega_rho, omega_rho, 1, 1, 1)
   and the forcing added with weight (1 - omega_i / 2), f* = (T^T)^{-1} k* by Gaussian elimination;
8. BGK of g, Eq. (7);
9. streaming, Eqs. (4)-(5), in the push form: f_i(x + c_i) <- f*_i(x), periodic in x (and in y
   without walls); a link leaving through a wall returns to its node in the opposite direction
   (half-way bounce-back), with the moving-wall term 2 w_j (c_j . U) / c_s^2 times 1 (f) or the
   node's new phi (g) on the returning links (reading R19).

Population arrays are nested lists P[i][y][x] of Fractions (post-streaming values).
"""
from __future__ import annotations

from fractions import Fraction as Q

CX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
CY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
W = [Q(4, 9)] + [Q(1, 9)] * 4 + [Q(1, 36)] * 4
CS2 = Q(1, 3)
WXX = [Q(0), Q(1, 3), Q(-1, 6), Q(1, 3), Q(-1, 6), Q(-1, 24), Q(-1, 24), Q(-1, 24), Q(-1, 24)]
WYY = [Q(0), Q(-1, 6), Q(1, 3), Q(-1, 6), Q(1, 3), Q(-1, 24), Q(-1, 24), Q(-1, 24), Q(-1, 24)]
WXY = [Q(0), Q(0), Q(0), Q(0), Q(0), Q(1, 4), Q(-1, 4), Q(1, 4), Q(-1, 4)]
SX = [Q(0), Q(4, 12), Q(0), Q(-4, 12), Q(0), Q(1, 12), Q(-1, 12), Q(-1, 12), Q(1, 12)]
SY = [Q(0), Q(0), Q(4, 12), Q(0), Q(-4, 12), Q(1, 12), Q(1, 12), Q(-1, 12), Q(-1, 12)]
SL = [Q(-20, 6), Q(4, 6), Q(4, 6), Q(4, 6), Q(4, 6), Q(1, 6), Q(1, 6), Q(1, 6), Q(1, 6)]


class Phys:
    """Exact parameters (Fractions): a, gamma, mobility M, Gamma, nu_l, nu_g, omega3, force,
    walls (0/1), wall velocities along x and the wall gradient."""

    def __init__(self, a, gamma, mobility, Gamma, nu_l, nu_g, omega3=Q(1), fx=Q(0), fy=Q(0), walls=0,
                 u_bottom=Q(0), u_top=Q(0), wall_gradient=Q(0)):
        self.a, self.gamma, self.M, self.Gamma = Q(a), Q(gamma), Q(mobility), Q(Gamma)
        self.w_l = 1 / (Q(nu_l) / CS2 + Q(1, 2))
        self.w_g = 1 / (Q(nu_g) / CS2 + Q(1, 2))
        self.w3 = Q(omega3)
        self.w_phi = 1 / (self.M / (self.Gamma * CS2) + Q(1, 2))
        self.fx, self.fy = Q(fx), Q(fy)
        self.walls = walls
        self.u_bottom, self.u_top = Q(u_bottom), Q(u_top)
        self.wgrad = Q(wall_gradient)


def phi_plane(g, nx, ny):
    return [[sum(g[i][y][x] for i in range(9)) for x in range(nx)] for y in range(ny)]


def phi_at(phi, nx, ny, c, x, y):
    """phi at (x, y) with periodic x; beyond a wall the ghost row (wall row minus the gradient)."""
    x %= nx
    if c.walls:
        if y < 0:
            return phi[0][x] - c.wgrad
        if y >= ny:
            return phi[ny - 1][x] - c.wgrad
    return phi[y % ny][x]


def stencils(phi, nx, ny, c, x, y):
    nb = [phi_at(phi, nx, ny, c, x + CX[i], y + CY[i]) for i in range(9)]
    dx = sum(SX[i] * nb[i] for i in range(9))
    dy = sum(SY[i] * nb[i] for i in range(9))
    lap = sum(SL[i] * nb[i] for i in range(9))
    return dx, dy, lap


def f_equilibrium(rho, ux, uy, pt, gamma, dx, dy):
    feq = [Q(0)] * 9
    u2 = ux * ux + uy * uy
    for i in range(1, 9):
        cu = CX[i] * ux + CY[i] * uy
        feq[i] = W[i] * (pt / CS2 + rho * (cu / CS2 + cu * cu / (2 * CS2 * CS2) - u2 / (2 * CS2))) + \
            gamma * (WXX[i] * dx * dx + WYY[i] * dy * dy + WXY[i] * dx * dy)
    feq[0] = rho - sum(feq[1:])
    return feq


def g_equilibrium(phi, mu, ux, uy, Gamma):
    geq = [Q(0)] * 9
    u2 = ux * ux + uy * uy
    for i in range(1, 9):
        cu = CX[i] * ux + CY[i] * uy
        geq[i] = W[i] * (Gamma * mu + phi * (cu / CS2 + cu * cu / (2 * CS2 * CS2) - u2 / (2 * CS2)))
    geq[0] = phi - sum(geq[1:])
    return geq


def basis_rows(ux, uy):
    """T^T: row j is the basis vector T_j of Eq. (15) over the directions, at c - v."""
    rows = []
    for j in range(9):
        r = []
        for i in range(9):
            bx, by = CX[i] - ux, CY[i] - uy
            r.append([Q(1), bx, by, bx * bx + by * by, bx * bx - by * by, bx * by, bx * bx * by, bx * by * by,
                      bx * bx * by * by][j])
        rows.append(r)
    return rows


def matvec(A, v):
    return [sum(A[j][i] * v[i] for i in range(9)) for j in range(9)]


def solve(A, b):
    """Exact Gaussian elimination of A x = b (first non-zero pivot)."""
    n = len(b)
    m = [list(A[r]) + [b[r]] for r in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if m[r][col] != 0)
        m[col], m[piv] = m[piv], m[col]
        for r in range(n):
            if r != col and m[r][col] != 0:
                fac = m[r][col] / m[col][col]
                m[r] = [m[r][k] - fac * m[col][k] for k in range(n + 1)]
    return [m[r][n] / m[r][r] for r in range(n)]


def guo_force(ux, uy, fx, fy):
    """Guo's forcing populations w_i [(c_i - v) / c_s^2 + (c_i . v) c_i / c_s^4] . F."""
    out = []
    for i in range(9):
        cu = CX[i] * ux + CY[i] * uy
        ex = (CX[i] - ux) / CS2 + cu * CX[i] / (CS2 * CS2)
        ey = (CY[i] - uy) / CS2 + cu * CY[i] / (CS2 * CS2)
        out.append(W[i] * (ex * fx + ey * fy))
    return out


def collide(f9, g9, phi, dx, dy, lap, c):
    """Post-collision (f*, g*) at one node."""
    rho = sum(f9)
    ux = (sum(f9[i] * CX[i] for i in range(9)) + c.fx / 2) / rho
    uy = (sum(f9[i] * CY[i] for i in range(9)) + c.fy / 2) / rho
    mu = c.a * (-phi + phi ** 3) - c.gamma * lap
    p0 = rho * CS2 + c.a * (-Q(1, 2) * phi ** 2 + Q(3, 4) * phi ** 4)
    pt = p0 - c.gamma * phi * lap
    w_rho = c.w_g + Q(1, 2) * (phi + 1) * (c.w_l - c.w_g)
    T = basis_rows(ux, uy)
    k = matvec(T, f9)
    keq = matvec(T, f_equilibrium(rho, ux, uy, pt, c.gamma, dx, dy))
    R = matvec(T, guo_force(ux, uy, c.fx, c.fy))
    rates = [Q(1), Q(1), Q(1), c.w3, w_rho, w_rho, Q(1), Q(1), Q(1)]
    ks = [k[j] + rates[j] * (keq[j] - k[j]) + (1 - rates[j] / 2) * R[j] for j in range(9)]
    fs = solve(T, ks)
    geq = g_equilibrium(phi, mu, ux, uy, c.Gamma)
    gs = [g9[i] + c.w_phi * (geq[i] - g9[i]) for i in range(9)]
    return fs, gs


def step(f, g, nx, ny, c):
    """One time step of the post-streaming populations (f, g) -> new (f, g)."""
    phi = phi_plane(g, nx, ny)
    fs = [[[None] * nx for _ in range(ny)] for _ in range(9)]
    gs = [[[None] * nx for _ in range(ny)] for _ in range(9)]
    for y in range(ny):
        for x in range(nx):
            dx, dy, lap = stencils(phi, nx, ny, c, x, y)
            a, b = collide([f[i][y][x] for i in range(9)], [g[i][y][x] for i in range(9)], phi[y][x], dx, dy, lap, c)
            for i in range(9):
                fs[i][y][x], gs[i][y][x] = a[i], b[i]
    fn = [[[None] * nx for _ in range(ny)] for _ in range(9)]
    gn = [[[None] * nx for _ in range(ny)] for _ in range(9)]
    for i in range(9):
        for y in range(ny):
            for x in range(nx):
                yd, xd = y + CY[i], (x + CX[i]) % nx
                if c.walls and not 0 <= yd < ny:
                    fn[OPP[i]][y][x], gn[OPP[i]][y][x] = fs[i][y][x], gs[i][y][x]
                else:
                    fn[i][yd % ny][xd], gn[i][yd % ny][xd] = fs[i][y][x], gs[i][y][x]
    if c.walls:  # moving walls: the links returning from the bottom (5, 6) and top (7, 8) wall
        for y, U, links in ((0, c.u_bottom, (5, 6)), (ny - 1, c.u_top, (7, 8))):
            if U == 0:
                continue
            for x in range(nx):
                ph = sum(gn[i][y][x] for i in range(9))
                for j in links:
                    t = 2 * W[j] * (CX[j] * U) / CS2
                    fn[j][y][x] += t
                    gn[j][y][x] += ph * t
    return fn, gn


def init(phi0, nx, ny, c):
    """Equilibrium populations of (phi0, rho = 1, v = 0) with the stencils of phi0 (reading R10)."""
    f = [[[None] * nx for _ in range(ny)] for _ in range(9)]
    g = [[[None] * nx for _ in range(ny)] for _ in range(9)]
    for y in range(ny):
        for x in range(nx):
            ph = phi0[y][x]
            dx, dy, lap = stencils(phi0, nx, ny, c, x, y)
            mu = c.a * (-ph + ph ** 3) - c.gamma * lap
            pt = CS2 + c.a * (-Q(1, 2) * ph ** 2 + Q(3, 4) * ph ** 4) - c.gamma * ph * lap
            fe = f_equilibrium(Q(1), Q(0), Q(0), pt, c.gamma, dx, dy)
            ge = g_equilibrium(ph, mu, Q(0), Q(0), c.Gamma)
            for i in range(9):
                f[i][y][x], g[i][y][x] = fe[i], ge[i]
    return f, g
