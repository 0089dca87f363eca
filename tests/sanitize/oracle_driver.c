/* Test driver for the FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer: the
 * oracle source is compiled into this program (without OpenMP) and every entry point runs on
 * small lattices with ragged sizes, walls, force, moving and wetting walls and the three
 * collision modes.  Exit status 0 and finite fields mean no sanitizer report. */
#include <stdio.h>

#include "../../oracle/lbcm_oracle.c"

static int run_case(int nx, int ny, int walls, int collision)
{
    orc_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx;
    p.ny = ny;
    p.walls = walls;
    p.a = 0.04;
    p.gamma = 0.08;
    p.mobility = 0.1;
    p.Gamma = 1.0;
    p.nu_l = 0.1;
    p.nu_g = 0.02;
    p.omega3 = 1.0;
    p.force_x = 1e-5;
    p.force_y = -2e-6;
    p.wall_ux_bottom = walls ? -1e-3 : 0.0;
    p.wall_ux_top = walls ? 2e-3 : 0.0;
    p.wall_gradient = walls ? 0.05 : 0.0;
    p.collision = collision;
    if (orc_check(&p) != 0) return 1;
    const size_t N = (size_t)nx * ny;
    double *phi = malloc(N * sizeof(double)), *rho = malloc(N * sizeof(double)), *ux = malloc(N * sizeof(double)),
           *uy = malloc(N * sizeof(double)), *p0 = malloc(N * sizeof(double));
    double *f = malloc(9 * N * sizeof(double)), *g = malloc(9 * N * sizeof(double));
    double *f2 = malloc(9 * N * sizeof(double)), *g2 = malloc(9 * N * sizeof(double));
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const double r = sqrt((x - nx / 2.0) * (x - nx / 2.0) + (y - ny / 2.0) * (y - ny / 2.0));
            phi[(size_t)y * nx + x] = tanh((0.3 * (nx < ny ? nx : ny) - r) / 2.0);
            rho[(size_t)y * nx + x] = 1.0 + 0.01 * sin(0.3 * x);
            ux[(size_t)y * nx + x] = 0.01 * cos(0.2 * y);
            uy[(size_t)y * nx + x] = -0.005 * sin(0.4 * x);
        }
    int bad = orc_init(&p, phi, rho, ux, uy, f, g) != 0;
    bad |= orc_step(&p, f, g, f2, g2) != 0;
    bad |= orc_run(&p, f2, g2, 5) != 0;
    bad |= orc_fields(&p, f2, g2, phi, rho, ux, uy, p0) != 0;
    for (size_t i = 0; i < N; ++i) bad |= !isfinite(phi[i]) || !isfinite(rho[i]) || !isfinite(ux[i]) || !isfinite(p0[i]);
    free(phi), free(rho), free(ux), free(uy), free(p0), free(f), free(g), free(f2), free(g2);
    return bad;
}

int main(void)
{
    int bad = 0;
    const int sizes[][2] = {{1, 1}, {3, 2}, {17, 13}, {24, 20}};
    for (int s = 0; s < 4; ++s)
        for (int walls = 0; walls < 2; ++walls)
            for (int c = 0; c < 3; ++c) bad |= run_case(sizes[s][0], sizes[s][1], walls, c);
    printf(bad ? "oracle driver: FAILED\n" : "oracle driver: ok\n");
    return bad;
}
