/*
 * Memory and undefined-behaviour check of the CPU oracle (test infrastructure only).
 *
 * Built with gcc -fsanitize=address,undefined and run by the test suite: it drives every
 * oracle entry point over the geometries the tests use (flat walls, a curved obstacle,
 * open inlet/outlet columns, both wetting schemes and the surface-energy rule, and degenerate
 * lattices: one row of fluid between walls, an all-solid box, a 2-column open channel) and
 * exits non-zero on a sanitizer report or a non-finite mass.  The oracle source is included
 * as one translation unit so that its internal passes are checked as they are compiled.
 */
#include "lbm_oracle.c"

#include <stdio.h>

static orc_params base_params(int nx, int ny) {
    orc_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx;
    p.ny = ny;
    p.nu_r = p.nu_b = 1.0 / 6.0;
    p.sigma = 0.01;
    p.beta = 0.7;
    p.theta_deg = 60.0;
    p.s_e = 1.64;
    p.s_eps = 1.54;
    p.s_q = 1.9;
    p.rho0 = 1.0;
    p.eps = 1e-10;
    return p;
}

/* Run one case: walls on the first and last rows unless `box`, a solid disk when r_obst > 0,
 * a red disk of radius r_drop at (xd, yd), the rest blue.  Returns 0 if the mass stays finite. */
static int run_case(const char *name, orc_params p, int walls, double r_obst, double r_drop,
                    double xd, double yd, int all_solid, int steps) {
    const int nx = p.nx, ny = p.ny;
    const size_t nn = (size_t)nx * ny;
    uint8_t *solid = calloc(nn, 1);
    double *rr = calloc(nn, sizeof(double)), *rb = calloc(nn, sizeof(double));
    double *iu = calloc(ny, sizeof(double));
    for (int y = 0; y < ny; y++) {
        iu[y] = p.open_x ? 0.01 : 0.0;
        for (int x = 0; x < nx; x++) {
            const size_t i = (size_t)y * nx + x;
            int s = all_solid || (walls && (y == 0 || y == ny - 1));
            const double ox = x - nx / 2.0, oy = y - ny / 2.0;
            if (r_obst > 0 && ox * ox + oy * oy < r_obst * r_obst) s = 1;
            solid[i] = (uint8_t)s;
            const double dx = x - xd, dy = y - yd;
            const int red = dx * dx + dy * dy < r_drop * r_drop;
            rr[i] = red ? 1.0 : 0.0;
            rb[i] = red ? 0.0 : 1.0;
        }
    }
    orc_ctx *c = orc_create(&p, solid, NULL, iu, rr, rb);
    int bad = 0;
    if (!c) {
        fprintf(stderr, "%s: orc_create rejected the case\n", name);
        bad = 1;
    } else {
        orc_step(c, steps);
        double m[2];
        orc_mass(c, m);
        double *buf = malloc(18 * nn * sizeof(double));
        for (int w = 0; w < 12; w++) bad |= orc_fields(c, w, buf) != 0;
        orc_get_pops(c, buf);
        orc_set_pops(c, buf);
        orc_step(c, 1);
        uint8_t *cls = malloc(nn);
        orc_classes(c, cls);
        orc_wall_normals(c, buf);
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                double n2[2];
                orc_e8_normal(solid, nx, ny, p.open_x, x, y, n2);
            }
        orc_mass(c, m);
        if (!isfinite(m[0]) || !isfinite(m[1])) bad = 1;
        printf("%-28s steps %lld  mass R %.12g B %.12g%s\n", name, orc_step_count(c), m[0], m[1],
               bad ? "  FAILED" : "");
        free(cls);
        free(buf);
        orc_destroy(c);
    }
    free(solid);
    free(rr);
    free(rb);
    free(iu);
    return bad;
}

int main(void) {
    int bad = 0;
    orc_params p = base_params(48, 26);
    bad |= run_case("droplet, flat walls", p, 1, 0.0, 9.0, 20.3, 1.0, 0, 40);
    p.scheme = 1;
    bad |= run_case("droplet, scheme (b)", p, 1, 0.0, 9.0, 20.3, 1.0, 0, 40);
    p.scheme = 0;
    p.surface_energy = 1;
    bad |= run_case("droplet, surface energy", p, 1, 0.0, 9.0, 20.3, 1.0, 0, 40);
    orc_params q = base_params(40, 40);
    q.theta_deg = 120.0;
    bad |= run_case("droplet on a cylinder", q, 0, 8.0, 7.0, 20.0, 30.5, 0, 40);
    orc_params o = base_params(60, 18);
    o.open_x = 1;
    o.nu_r = 0.5;
    o.nu_b = 0.05;
    o.outlet_u = 0.01;
    bad |= run_case("open channel", o, 1, 0.0, 12.0, 0.0, 9.0, 0, 40);
    o.scheme = 1;
    bad |= run_case("open channel, scheme (b)", o, 1, 0.0, 12.0, 0.0, 9.0, 0, 40);
    orc_params t = base_params(2, 6);
    t.open_x = 1;
    bad |= run_case("2-column open channel", t, 1, 0.0, 1.5, 0.0, 3.0, 0, 10);
    bad |= run_case("one fluid row", base_params(16, 3), 1, 0.0, 2.0, 8.0, 1.0, 0, 10);
    bad |= run_case("all solid", base_params(8, 8), 0, 0.0, 0.0, 0.0, 0.0, 1, 5);
    bad |= run_case("1 x 1 periodic", base_params(1, 1), 0, 0.0, 0.5, 0.0, 0.0, 0, 5);

    /* the stand-alone routines */
    double f[9], g[9], o2[2], fr[9], fb[9];
    orc_feq(1.0, 0.05, -0.02, f);
    orc_guo(0.05, -0.02, 1e-4, 2e-4, g);
    bad |= orc_collide(&p, f, 1e-4, 2e-4, 0.3, g) != 0;
    orc_recolor(g, 0.6, 0.4, 0.6, 0.8, 0.7, fr, fb);
    orc_wet_correct(0.0, -1.0, 60.0, 1e-10, 0.3, 0.4, o2);
    orc_wet_correct(0.0, -1.0, 60.0, 1e-10, 0.0, 0.0, o2);
    const double phi[9] = {0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9};
    const uint8_t fl[9] = {1, 1, 0, 1, 1, 0, 1, 1, 0};
    orc_grad48(phi, fl, o2);
    double M[81], Mi[81];
    orc_matrices(M, Mi);
    int ex[9], ey[9], cx[24], cy[24];
    double w[9], w24[24];
    orc_lattice(ex, ey, w);
    bad |= orc_e8_table(cx, cy, w24) != 24;
    printf(bad ? "oracle sanitizer check FAILED\n" : "oracle sanitizer check passed\n");
    return bad;
}
