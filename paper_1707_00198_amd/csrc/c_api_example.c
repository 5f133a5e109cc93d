/*
 * The C interface used from plain C (C99, no Python, no torch): a static droplet on a flat wall.
 *
 *   lbm_c_example [f64|f32|f16|c16] [steps]
 *
 * A 64 x 32 lattice, periodic in x, with solid rows at y = 0 and y = 31; a red half-disc of
 * radius 10 on the bottom wall at x = 32 in blue fluid; prescribed contact angle 60 degrees.
 * The program sizes and allocates the device buffers itself (hipMalloc), creates a context on
 * the default stream, advances it, reads the red density back (lbm_read_fields into device
 * memory, then hipMemcpy) and prints the colour masses before and after and a few densities
 * with 17 significant digits, so that a caller can compare them with any other driver of the
 * same library.  Exit status 0 on success, 1 on a library error (its message is printed), 2
 * when no HIP device is usable.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbmcg.h"

enum { NX = 64, NY = 32 };

static int check(int status, const char *what) {
    if (status != LBM_OK) {
        fprintf(stderr, "%s failed (%d): %s\n", what, status, lbm_last_error());
        exit(1);
    }
    return status;
}

/* The set-up, shared by every storage: solid rows at y = 0 and NY - 1; red where the node
 * centre lies inside the circle of radius 10 about (32, 1) (the first fluid row is y = 1). */
static void make_droplet(uint8_t *solid, double *rho_r, double *rho_b) {
    for (int y = 0; y < NY; y++)
        for (int x = 0; x < NX; x++) {
            const int k = y * NX + x;
            const int wall = (y == 0 || y == NY - 1);
            const double dx = x - 32.0, dy = y - 1.0;
            const int red = !wall && dx * dx + dy * dy < 100.0;
            solid[k] = (uint8_t)wall;
            rho_r[k] = wall ? 0.0 : (red ? 1.0 : 0.0);
            rho_b[k] = wall ? 0.0 : (red ? 0.0 : 1.0);
        }
}

int main(int argc, char **argv) {
    const char *name = argc > 1 ? argv[1] : "f64";
    const long steps = argc > 2 ? atol(argv[2]) : 200;
    int storage = -1;
    const char *names[4] = {"f64", "f32", "f16", "c16"};
    for (int i = 0; i < 4; i++)
        if (strcmp(name, names[i]) == 0) storage = i;
    if (storage < 0 || steps < 0) {
        fprintf(stderr, "usage: %s [f64|f32|f16|c16] [steps]\n", argv[0]);
        return 1;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        fprintf(stderr, "no HIP device is available\n");
        return 2;
    }

    static uint8_t solid[NX * NY];
    static double rho_r[NX * NY], rho_b[NX * NY];
    make_droplet(solid, rho_r, rho_b);

    lbm_domain_desc d;
    memset(&d, 0, sizeof d);
    d.nx = NX;
    d.ny = NY;
    d.open_x = 0;
    d.wetting = 0;
    d.solid = solid;
    d.ns = NULL; /* wall normal from the eighth-order stencil (Eqs. 32-33) */
    d.inlet_ux = NULL;
    d.rho_r0 = rho_r;
    d.rho_b0 = rho_b;
    d.nu_r = d.nu_b = 1.0 / 6.0;
    d.sigma = 0.01;
    d.beta = 0.7;
    d.theta_deg = 60.0;
    d.s_e = 1.64;
    d.s_eps = 1.54;
    d.s_q = 1.9;
    d.rho0 = 1.0;
    d.eps = 1e-10;
    d.outlet_u = 0.0;

    size_t state_bytes = 0, scratch_bytes = 0;
    check(lbm_query_bytes(&d, 1, storage, &state_bytes, &scratch_bytes), "lbm_query_bytes");
    void *state = NULL, *scratch = NULL;
    double *field = NULL;
    if (hipMalloc(&state, state_bytes) != hipSuccess || hipMalloc(&scratch, scratch_bytes) != hipSuccess ||
        hipMalloc((void **)&field, sizeof(double) * NX * NY) != hipSuccess) {
        fprintf(stderr, "hipMalloc failed\n");
        return 2;
    }
    lbm_ctx *ctx = NULL;
    check(lbm_create(&d, 1, storage, state, state_bytes, scratch, scratch_bytes, NULL, &ctx), "lbm_create");

    double m0[2], m1[2];
    check(lbm_mass(ctx, m0), "lbm_mass");
    check(lbm_step(ctx, steps), "lbm_step");
    check(lbm_mass(ctx, m1), "lbm_mass");
    check(lbm_read_fields(ctx, 0, LBM_FIELD_RHO_R, field, (size_t)NX * NY), "lbm_read_fields");
    static double host[NX * NY];
    if (hipMemcpy(host, field, sizeof host, hipMemcpyDeviceToHost) != hipSuccess) {
        fprintf(stderr, "hipMemcpy failed\n");
        return 1;
    }
    printf("storage %s steps %lld\n", name, (long long)lbm_steps_taken(ctx));
    printf("mass_before %.17g %.17g\n", m0[0], m0[1]);
    printf("mass_after %.17g %.17g\n", m1[0], m1[1]);
    const int samples[4][2] = {{32, 1}, {32, 8}, {40, 5}, {10, 20}};
    for (int i = 0; i < 4; i++) {
        const int x = samples[i][0], y = samples[i][1];
        printf("rho_r %d %d %.17g\n", x, y, host[y * NX + x]);
    }
    lbm_destroy(ctx);
    hipFree(field);
    hipFree(scratch);
    hipFree(state);
    return 0;
}
