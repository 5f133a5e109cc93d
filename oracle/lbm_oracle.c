/*
 * Plain FP64 CPU oracle for one time step of the two-colour D2Q9 lattice Boltzmann
 * method with the improved geometric wetting boundary of Yu, Liu, Zhang and Liang,
 * "Lattice Boltzmann simulation of viscous fingering of immiscible displacement in a
 * channel using an improved wetting scheme" (arXiv:1707.00198).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code with the GPU library.
 *
 * Storage is the literal form of the paper: two population sets f_{alpha,R}, f_{alpha,B}
 * per node (Sec. II A), indexed pop[(k*9 + alpha)*nn + y*nx + x], k = 0 red, 1 blue.
 * Every stage of a step is a separate pass over the whole lattice, in the order
 *   densities (Eqs. 16, 12) -> virtual rho^N on outermost solid nodes (Eq. 29)
 *   -> colour gradient (Eq. 28) -> wetting correction on outermost fluid nodes
 *   (Eqs. 30-36) -> interface normals (Eq. 22) and virtual normals (Eq. 29, second BC)
 *   -> curvature (Eq. 13), CSF force (Eq. 10), velocity (Eq. 17), viscosity (Eqs. 18, 5)
 *   -> MRT collision with Guo forcing (Eqs. 1-9) -> recolouring (Eq. 14)
 *   -> streaming with half-way bounce-back (Eq. 15) -> open-boundary completion.
 * Each pass reads only arrays completed by earlier passes.
 *
 * Two per-lattice options give the wetting variants the paper compares (Sec. III A):
 *  - scheme (b) of Sec. III A 2: no virtual normals on outermost solid nodes; the
 *    normal derivatives on outermost fluid nodes come from the one-sided mean of
 *    Eq. 48 over the directions whose neighbour is fluid (Eq. 28 everywhere else);
 *  - the surface-energy rule of Sec. III A 1: the virtual rho^N on outermost solid
 *    nodes is cos(theta) instead of Eq. 29, and the colour gradient is not corrected
 *    (no Eqs. 30-36).
 * They are independent; the surface-energy model of the comparison in Fig. 2 has no
 * zero-interface-force condition, i.e. it is the surface-energy rule with scheme (b).
 *
 * Readings of passages that are garbled or silent (each is listed in the design notes):
 *  - Eq. 3, last row: printed as 0 0 0 0 0 1 1 1 -1, which is not orthogonal to the
 *    others; the p_xy = e_x e_y row 0 0 0 0 0 1 -1 1 -1 is used.
 *  - Eq. 14: the blue line is printed with "+beta"; Latva-Kokko/Rothman recolouring has
 *    "-beta" for blue, which is what makes the two colours sum to f'.
 *  - Eq. 15: right-hand side read as f''_{alpha,k}.
 *  - Eq. 5: nu is the kinematic viscosity; Eq. 18 is applied to nu with equal densities.
 *  - n = 0 (and no recolouring perturbation) where |grad rho^N| <= eps.
 *  - The wall normal points into the solid; Eq. 34 is a counter-clockwise rotation by
 *    +theta for (n_f)_1 and by -theta for (n_f)_2; a tie D1 == D2 picks (n_f)_1.
 *  - "Outermost" nodes use the D2Q9 8-neighbourhood; Eq. 29 sums over alpha = 1..8.
 *  - Eq. 48: alpha_1 runs over 1..8 with a fluid neighbour (the rest direction is in
 *    neither sum), and the e_{alpha i} of its numerator is read as e_{alpha_1 i}.
 *  - Stencils wrap periodically in y always, in x when x is periodic; with an open x
 *    axis, stencil accesses beyond x = 0 or x = nx-1 are clamped to the edge column, and
 *    the eighth-order wall-normal stencil counts nodes beyond an open edge as fluid.
 *  - Open x boundaries: Zou-He velocity inlet at x = 0 (unknowns alpha = 1, 5, 8 of the
 *    total f, coloured pure red) and a convective outlet at x = nx-1
 *    (f_a <- [f_a(t) + U f_a(x-1, t+1)] / (1 + U) for alpha = 3, 6, 7, coloured with
 *    the outlet node's own red fraction rho_R/rho of the step).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, ny;     /* lattice extent including solid nodes */
    int32_t open_x;     /* 0: periodic in x; 1: inlet at x = 0, outlet at x = nx-1 */
    int32_t scheme;     /* 0: scheme (a) of Sec. III A 2 (virtual normals, Eq. 29);
                           1: scheme (b) (Eq. 48 on outermost fluid nodes) */
    double nu_r, nu_b;  /* kinematic viscosities of red and blue */
    double sigma;       /* interfacial tension coefficient (Eq. 10) */
    double beta;        /* segregation parameter (Eq. 14) */
    double theta_deg;   /* prescribed contact angle, measured in the red phase */
    double s_e, s_eps, s_q; /* relaxation rates of e, epsilon and q moments (Eq. 6) */
    double rho0;        /* reference density (unity) */
    double eps;         /* |grad rho^N| threshold below which n = 0 */
    double outlet_u;    /* convective velocity of the outlet condition */
    double body_fx, body_fy; /* uniform body force added to F; a test hook, zero in the paper */
    int32_t surface_energy;  /* 0: Eq. 29 and Eqs. 30-36; 1: rho^N = cos(theta) on outermost
                                solid nodes, uncorrected gradient (Sec. III A 1) */
} orc_params;

/* D2Q9 velocities in the paper's numbering (Sec. II A, after Eq. 7). */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

/* Transformation matrix of Eq. 3 with the corrected last row. */
static const double MROW[81] = {
     1,  1,  1,  1,  1,  1,  1,  1,  1,
    -4, -1, -1, -1, -1,  2,  2,  2,  2,
     4, -2, -2, -2, -2,  1,  1,  1,  1,
     0,  1,  0, -1,  0,  1, -1, -1,  1,
     0, -2,  0,  2,  0,  1, -1, -1,  1,
     0,  0,  1,  0, -1,  1,  1, -1, -1,
     0,  0, -2,  0,  2,  1,  1, -1, -1,
     0,  1, -1,  1, -1,  0,  0,  0,  0,
     0,  0,  0,  0,  0,  1, -1,  1, -1};

enum { CLS_FLUID = 0, CLS_FLUID_BND = 1, CLS_SOLID_BND = 2, CLS_SOLID = 3 };

typedef struct orc_ctx {
    orc_params p;
    int nx, ny;
    size_t nn;
    uint8_t *solid;
    uint8_t *cls;
    double *ns;        /* 2*nn: wall normal (into the solid) at outermost fluid nodes */
    double *inlet_ux;  /* ny: prescribed inlet velocity per row */
    double *f, *fn, *fpost; /* 18*nn each */
    double *rhoR, *rhoB, *rhoN, *gx, *gy, *nvx, *nvy, *kap, *Fx, *Fy, *ux, *uy;
    double Minv[81];
    long long step;
} orc_ctx;

/* ------------------------------------------------------------------ helpers */

static int wrap_y(const orc_ctx *c, int y) { return ((y % c->ny) + c->ny) % c->ny; }

/* Stencil neighbour column: periodic wrap, or clamp at an open x axis. */
static int stencil_x(const orc_ctx *c, int x) {
    if (!c->p.open_x) return ((x % c->nx) + c->nx) % c->nx;
    if (x < 0) return 0;
    if (x >= c->nx) return c->nx - 1;
    return x;
}

static size_t nb_index(const orc_ctx *c, int x, int y, int a) {
    int xn = stencil_x(c, x + EX[a]);
    int yn = wrap_y(c, y + EY[a]);
    return (size_t)yn * c->nx + xn;
}

/* Gauss-Jordan inverse with partial pivoting; returns 0 on success. */
static int invert9(const double *A, double *Ainv) {
    double a[9][18];
    for (int i = 0; i < 9; i++)
        for (int j = 0; j < 18; j++)
            a[i][j] = j < 9 ? A[i * 9 + j] : (j - 9 == i ? 1.0 : 0.0);
    for (int col = 0; col < 9; col++) {
        int piv = col;
        for (int r = col + 1; r < 9; r++)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (fabs(a[piv][col]) < 1e-14) return -1;
        if (piv != col)
            for (int j = 0; j < 18; j++) {
                double t = a[col][j];
                a[col][j] = a[piv][j];
                a[piv][j] = t;
            }
        double d = a[col][col];
        for (int j = 0; j < 18; j++) a[col][j] /= d;
        for (int r = 0; r < 9; r++) {
            if (r == col) continue;
            double m = a[r][col];
            if (m != 0.0)
                for (int j = 0; j < 18; j++) a[r][j] -= m * a[col][j];
        }
    }
    for (int i = 0; i < 9; i++)
        for (int j = 0; j < 9; j++) Ainv[i * 9 + j] = a[i][j + 9];
    return 0;
}

static void matvec9(const double *A, const double *x, double *y) {
    for (int i = 0; i < 9; i++) {
        double s = 0.0;
        for (int j = 0; j < 9; j++) s += A[i * 9 + j] * x[j];
        y[i] = s;
    }
}

/* -------------------------------------------------- single-node building blocks */

/* Eq. 7 with c_s^2 = 1/3. */
void orc_feq(double rho, double ux, double uy, double *out) {
    double uu = ux * ux + uy * uy;
    for (int a = 0; a < 9; a++) {
        double eu = EX[a] * ux + EY[a] * uy;
        out[a] = rho * W[a] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
}

/* Eq. 9 (Guo forcing in velocity space), delta_t = 1. */
void orc_guo(double ux, double uy, double Fx, double Fy, double *out) {
    for (int a = 0; a < 9; a++) {
        double eu = EX[a] * ux + EY[a] * uy;
        double cx = 3.0 * (EX[a] - ux) + 9.0 * eu * EX[a];
        double cy = 3.0 * (EY[a] - uy) + 9.0 * eu * EY[a];
        out[a] = W[a] * (cx * Fx + cy * Fy);
    }
}

/* Local relaxation rate of the shear moments from Eqs. 18 and 5. */
static double shear_rate(const orc_params *p, double rhoN) {
    double inv_nu = (1.0 + rhoN) / (2.0 * p->nu_r) + (1.0 - rhoN) / (2.0 * p->nu_b);
    double nu = 1.0 / inv_nu;
    double tau = 3.0 * nu + 0.5;
    return 1.0 / tau;
}

/* MRT collision with forcing, Eqs. 1, 2, 8: returns the post-collision total f'.
 * u is the force-corrected velocity of Eq. 17. */
static void collide_node(const orc_params *p, const double *Minv, const double *f,
                         double rho, double ux, double uy, double Fx, double Fy,
                         double rhoN, double *fout) {
    double feq[9], ft[9], m[9], meq[9], mf[9], ms[9];
    double sv = shear_rate(p, rhoN);
    double S[9] = {1.0, p->s_e, p->s_eps, 1.0, p->s_q, 1.0, p->s_q, sv, sv};
    orc_feq(rho, ux, uy, feq);
    orc_guo(ux, uy, Fx, Fy, ft);
    matvec9(MROW, f, m);
    matvec9(MROW, feq, meq);
    matvec9(MROW, ft, mf);
    for (int k = 0; k < 9; k++)
        ms[k] = m[k] - S[k] * (m[k] - meq[k]) + (1.0 - 0.5 * S[k]) * mf[k];
    matvec9(Minv, ms, fout);
}

/* Exposed for unit checks: one collision of a total distribution f with force F and
 * colour indicator rhoN (which sets the local viscosity). */
int orc_collide(const orc_params *p, const double *f, double Fx, double Fy, double rhoN,
                double *fout) {
    double Minv[81];
    if (invert9(MROW, Minv)) return -1;
    double rho = 0, jx = 0, jy = 0;
    for (int a = 0; a < 9; a++) {
        rho += f[a];
        jx += f[a] * EX[a];
        jy += f[a] * EY[a];
    }
    double ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho;
    collide_node(p, Minv, f, rho, ux, uy, Fx, Fy, rhoN, fout);
    return 0;
}

/* Eq. 14 (with the blue sign read as minus). n is the unit interface normal or 0. */
void orc_recolor(const double *fp, double rR, double rB, double nx, double ny, double beta,
                 double *outR, double *outB) {
    double rho = rR + rB;
    for (int a = 0; a < 9; a++) {
        double pert = beta * (rR * rB / rho) * W[a] * (EX[a] * nx + EY[a] * ny);
        outR[a] = (rR / rho) * fp[a] + pert;
        outB[a] = (rB / rho) * fp[a] - pert;
    }
}

/* Eqs. 30-36: corrected colour gradient on an outermost fluid node. */
void orc_wet_correct(double nsx, double nsy, double theta_deg, double eps, double gx,
                     double gy, double *out) {
    double g = sqrt(gx * gx + gy * gy);
    if (!(g > eps)) {
        out[0] = gx;
        out[1] = gy;
        return;
    }
    double ex = gx / g, ey = gy / g; /* Eq. 30 */
    double th = theta_deg * M_PI / 180.0;
    double ct = cos(th), st = sin(th);
    /* Eq. 34: row vector n_s times the rotation matrix, for +theta and -theta. */
    double n1x = nsx * ct - nsy * st, n1y = nsx * st + nsy * ct;
    double n2x = nsx * ct + nsy * st, n2y = -nsx * st + nsy * ct;
    double d1 = sqrt((n1x - ex) * (n1x - ex) + (n1y - ey) * (n1y - ey)); /* Eq. 35 */
    double d2 = sqrt((n2x - ex) * (n2x - ex) + (n2y - ey) * (n2y - ey));
    if (d1 <= d2) { /* Eq. 36 */
        out[0] = g * n1x; /* Eq. 31 */
        out[1] = g * n1y;
    } else {
        out[0] = g * n2x;
        out[1] = g * n2y;
    }
}

/* Eq. 48: one-sided gradient at an outermost fluid node.  phi9[a] is phi at x + e_a
 * (phi9[0] = phi(x)), fluid9[a] says whether that neighbour is fluid; the sums run over the
 * directions a = 1..8 into fluid. */
void orc_grad48(const double *phi9, const uint8_t *fluid9, double *out) {
    double sx = 0.0, sy = 0.0, den = 0.0;
    for (int a = 1; a < 9; a++) {
        if (!fluid9[a]) continue;
        double diff = phi9[a] - phi9[0];
        sx += W[a] * diff * EX[a];
        sy += W[a] * diff * EY[a];
        den += W[a];
    }
    out[0] = sx / den;
    out[1] = sy / den;
}

/* Eighth-order isotropic stencil of Eqs. 32-33: 24 vectors and weights. */
static int e8_cx[24], e8_cy[24];
static double e8_w[24];
static int e8_ready = 0;

static void e8_build(void) {
    if (e8_ready) return;
    int n = 0;
    for (int cy = -2; cy <= 2; cy++)
        for (int cx = -2; cx <= 2; cx++) {
            int r2 = cx * cx + cy * cy;
            double w = 0.0;
            if (r2 == 1) w = 4.0 / 21.0;
            else if (r2 == 2) w = 4.0 / 45.0;
            else if (r2 == 4) w = 1.0 / 60.0;
            else if (r2 == 5) w = 2.0 / 315.0;
            else if (r2 == 8) w = 1.0 / 5040.0;
            if (w == 0.0) continue;
            e8_cx[n] = cx;
            e8_cy[n] = cy;
            e8_w[n] = w;
            n++;
        }
    e8_ready = 1;
}

int orc_e8_table(int *cx, int *cy, double *w) {
    e8_build();
    for (int k = 0; k < 24; k++) {
        cx[k] = e8_cx[k];
        cy[k] = e8_cy[k];
        w[k] = e8_w[k];
    }
    return 24;
}

/* Eq. 32 at node (x, y) of a solid indicator field. */
void orc_e8_normal(const uint8_t *solid, int nx, int ny, int open_x, int x, int y,
                   double *out) {
    e8_build();
    double sx = 0.0, sy = 0.0;
    for (int k = 0; k < 24; k++) {
        int xx = x + e8_cx[k], yy = ((y + e8_cy[k]) % ny + ny) % ny;
        int s;
        if (open_x && (xx < 0 || xx >= nx)) {
            s = 0;
        } else {
            xx = ((xx % nx) + nx) % nx;
            s = solid[(size_t)yy * nx + xx] ? 1 : 0;
        }
        sx += e8_w[k] * s * e8_cx[k];
        sy += e8_w[k] * s * e8_cy[k];
    }
    double m = sqrt(sx * sx + sy * sy);
    if (m > 0.0) {
        out[0] = sx / m;
        out[1] = sy / m;
    } else {
        out[0] = 0.0;
        out[1] = 0.0;
    }
}

/* ---------------------------------------------------------------- context */

void orc_destroy(orc_ctx *c) {
    if (!c) return;
    free(c->solid); free(c->cls); free(c->ns); free(c->inlet_ux);
    free(c->f); free(c->fn); free(c->fpost);
    free(c->rhoR); free(c->rhoB); free(c->rhoN); free(c->gx); free(c->gy);
    free(c->nvx); free(c->nvy); free(c->kap); free(c->Fx); free(c->Fy);
    free(c->ux); free(c->uy);
    free(c);
}

/* solid: nx*ny (1 = solid).  ns: optional 2*nx*ny analytic wall normals (into the
 * solid), NULL selects Eq. 32.  inlet_ux: ny values (used when open_x).
 * rho_r0, rho_b0: initial densities; populations start at rho_k w_alpha (u = 0). */
orc_ctx *orc_create(const orc_params *p, const uint8_t *solid, const double *ns,
                    const double *inlet_ux, const double *rho_r0, const double *rho_b0) {
    if (p->nx < 1 || p->ny < 1 || (p->open_x && p->nx < 2)) return NULL;
    if ((p->scheme != 0 && p->scheme != 1) || (p->surface_energy != 0 && p->surface_energy != 1))
        return NULL;
    orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    c->p = *p;
    c->nx = p->nx;
    c->ny = p->ny;
    c->nn = (size_t)p->nx * p->ny;
    size_t nn = c->nn;
    c->solid = (uint8_t *)malloc(nn);
    c->cls = (uint8_t *)malloc(nn);
    c->ns = (double *)calloc(2 * nn, sizeof(double));
    c->inlet_ux = (double *)calloc(c->ny, sizeof(double));
    c->f = (double *)calloc(18 * nn, sizeof(double));
    c->fn = (double *)calloc(18 * nn, sizeof(double));
    c->fpost = (double *)calloc(18 * nn, sizeof(double));
    double **fields[] = {&c->rhoR, &c->rhoB, &c->rhoN, &c->gx, &c->gy, &c->nvx,
                         &c->nvy, &c->kap, &c->Fx, &c->Fy, &c->ux, &c->uy};
    for (int i = 0; i < 12; i++) *fields[i] = (double *)calloc(nn, sizeof(double));
    if (invert9(MROW, c->Minv)) {
        orc_destroy(c);
        return NULL;
    }
    for (size_t i = 0; i < nn; i++) c->solid[i] = solid[i] ? 1 : 0;
    if (inlet_ux) memcpy(c->inlet_ux, inlet_ux, c->ny * sizeof(double));

    /* Node classes (D2Q9 8-neighbourhood). */
    for (int y = 0; y < c->ny; y++)
        for (int x = 0; x < c->nx; x++) {
            size_t i = (size_t)y * c->nx + x;
            int any_other = 0;
            for (int a = 1; a < 9; a++) {
                size_t j = nb_index(c, x, y, a);
                if (c->solid[j] != c->solid[i]) any_other = 1;
            }
            if (c->solid[i]) c->cls[i] = any_other ? CLS_SOLID_BND : CLS_SOLID;
            else c->cls[i] = any_other ? CLS_FLUID_BND : CLS_FLUID;
        }

    /* Wall normals on outermost fluid nodes: analytic if given, else Eq. 32. */
    for (int y = 0; y < c->ny; y++)
        for (int x = 0; x < c->nx; x++) {
            size_t i = (size_t)y * c->nx + x;
            if (c->cls[i] != CLS_FLUID_BND) continue;
            double v[2];
            if (ns) {
                double m = sqrt(ns[2 * i] * ns[2 * i] + ns[2 * i + 1] * ns[2 * i + 1]);
                v[0] = m > 0 ? ns[2 * i] / m : 0.0;
                v[1] = m > 0 ? ns[2 * i + 1] / m : 0.0;
            } else {
                orc_e8_normal(c->solid, c->nx, c->ny, c->p.open_x, x, y, v);
            }
            c->ns[2 * i] = v[0];
            c->ns[2 * i + 1] = v[1];
        }

    for (size_t i = 0; i < nn; i++) {
        if (c->solid[i]) continue;
        for (int a = 0; a < 9; a++) {
            c->f[(0 * 9 + a) * nn + i] = rho_r0[i] * W[a];
            c->f[(1 * 9 + a) * nn + i] = rho_b0[i] * W[a];
        }
    }
    return c;
}

/* ------------------------------------------------------------ step passes */

static void pass_density(orc_ctx *c) {
    size_t nn = c->nn;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < (long)nn; i++) {
        if (c->solid[i]) {
            c->rhoR[i] = c->rhoB[i] = c->rhoN[i] = 0.0;
            continue;
        }
        double rR = 0.0, rB = 0.0;
        for (int a = 0; a < 9; a++) {
            rR += c->f[(0 * 9 + a) * nn + i]; /* Eq. 16 */
            rB += c->f[(1 * 9 + a) * nn + i];
        }
        c->rhoR[i] = rR;
        c->rhoB[i] = rB;
        c->rhoN[i] = (rR - rB) / (rR + rB); /* Eq. 12 */
    }
}

/* Eq. 29 on the outermost solid nodes: weighted mean over fluid neighbours. */
static void pass_virtual(orc_ctx *c, double *phi) {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < c->ny; y++)
        for (int x = 0; x < c->nx; x++) {
            size_t i = (size_t)y * c->nx + x;
            if (c->cls[i] != CLS_SOLID_BND) continue;
            double num = 0.0, den = 0.0;
            for (int a = 1; a < 9; a++) {
                size_t j = nb_index(c, x, y, a);
                if (c->solid[j]) continue;
                num += W[a] * phi[j];
                den += W[a];
            }
            phi[i] = num / den;
        }
}

/* Surface-energy rule: rho^N = cos(theta) on the outermost solid nodes. */
static void pass_surface_energy(orc_ctx *c) {
    double v = cos(c->p.theta_deg * M_PI / 180.0);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < (long)c->nn; i++)
        if (c->cls[i] == CLS_SOLID_BND) c->rhoN[i] = v;
}

/* Eq. 28 at fluid node (x, y) of field phi (solid neighbours hold virtual values). */
static void iso_gradient(const orc_ctx *c, const double *phi, int x, int y, double *gx,
                         double *gy) {
    double sx = 0.0, sy = 0.0;
    for (int a = 1; a < 9; a++) {
        double v = phi[nb_index(c, x, y, a)];
        sx += W[a] * v * EX[a];
        sy += W[a] * v * EY[a];
    }
    *gx = 3.0 * sx;
    *gy = 3.0 * sy;
}

static void pass_gradient(orc_ctx *c) {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < c->ny; y++)
        for (int x = 0; x < c->nx; x++) {
            size_t i = (size_t)y * c->nx + x;
            if (c->solid[i]) {
                c->gx[i] = c->gy[i] = 0.0;
                continue;
            }
            iso_gradient(c, c->rhoN, x, y, &c->gx[i], &c->gy[i]);
        }
}

static void pass_wetting(orc_ctx *c) {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < (long)c->nn; i++) {
        if (c->cls[i] != CLS_FLUID_BND) continue;
        double out[2];
        orc_wet_correct(c->ns[2 * i], c->ns[2 * i + 1], c->p.theta_deg, c->p.eps, c->gx[i],
                        c->gy[i], out);
        c->gx[i] = out[0];
        c->gy[i] = out[1];
    }
}

static void pass_normals(orc_ctx *c) {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < (long)c->nn; i++) {
        if (c->solid[i]) {
            c->nvx[i] = c->nvy[i] = 0.0;
            continue;
        }
        double g = sqrt(c->gx[i] * c->gx[i] + c->gy[i] * c->gy[i]);
        if (g > c->p.eps) { /* Eq. 22 */
            c->nvx[i] = c->gx[i] / g;
            c->nvy[i] = c->gy[i] / g;
        } else {
            c->nvx[i] = c->nvy[i] = 0.0;
        }
    }
    /* Second boundary condition of scheme (a): virtual normals on outermost solid nodes
     * (Eq. 29).  Scheme (b) leaves them 0; no stencil reads them then. */
    if (c->p.scheme == 0) {
        pass_virtual(c, c->nvx);
        pass_virtual(c, c->nvy);
    }
}

/* Eq. 48 at outermost fluid node (x, y) of field phi. */
static void one_sided_gradient(const orc_ctx *c, const double *phi, int x, int y, double *gx,
                               double *gy) {
    double phi9[9], out[2];
    uint8_t fluid9[9];
    phi9[0] = phi[(size_t)y * c->nx + x];
    fluid9[0] = 1;
    for (int a = 1; a < 9; a++) {
        size_t j = nb_index(c, x, y, a);
        phi9[a] = phi[j];
        fluid9[a] = !c->solid[j];
    }
    orc_grad48(phi9, fluid9, out);
    *gx = out[0];
    *gy = out[1];
}

/* Curvature (Eq. 13), CSF force (Eq. 10) and force-corrected velocity (Eq. 17). */
static void pass_force(orc_ctx *c) {
    size_t nn = c->nn;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < c->ny; y++)
        for (int x = 0; x < c->nx; x++) {
            size_t i = (size_t)y * c->nx + x;
            if (c->solid[i]) {
                c->kap[i] = c->Fx[i] = c->Fy[i] = c->ux[i] = c->uy[i] = 0.0;
                continue;
            }
            double dnxdx, dnxdy, dnydx, dnydy;
            if (c->p.scheme == 1 && c->cls[i] == CLS_FLUID_BND) {
                one_sided_gradient(c, c->nvx, x, y, &dnxdx, &dnxdy);
                one_sided_gradient(c, c->nvy, x, y, &dnydx, &dnydy);
            } else {
                iso_gradient(c, c->nvx, x, y, &dnxdx, &dnxdy);
                iso_gradient(c, c->nvy, x, y, &dnydx, &dnydy);
            }
            double nx = c->nvx[i], ny = c->nvy[i];
            double kappa = -nx * nx * dnydy - ny * ny * dnxdx + nx * ny * (dnxdy + dnydx);
            double Fx = 0.5 * c->p.sigma * kappa * c->gx[i] + c->p.body_fx;
            double Fy = 0.5 * c->p.sigma * kappa * c->gy[i] + c->p.body_fy;
            double jx = 0.0, jy = 0.0;
            for (int k = 0; k < 2; k++)
                for (int a = 0; a < 9; a++) {
                    double fa = c->f[(k * 9 + a) * nn + i];
                    jx += fa * EX[a];
                    jy += fa * EY[a];
                }
            double rho = c->rhoR[i] + c->rhoB[i];
            c->kap[i] = kappa;
            c->Fx[i] = Fx;
            c->Fy[i] = Fy;
            c->ux[i] = (jx + 0.5 * Fx) / rho;
            c->uy[i] = (jy + 0.5 * Fy) / rho;
        }
}

/* Everything before the collision: leaves rhoN, grad, n, kappa, F and u for the
 * current populations in the context. */
static void prepare(orc_ctx *c) {
    pass_density(c);
    if (c->p.surface_energy)
        pass_surface_energy(c);
    else
        pass_virtual(c, c->rhoN);
    pass_gradient(c);
    if (!c->p.surface_energy) pass_wetting(c);
    pass_normals(c);
    pass_force(c);
}

static void pass_collide(orc_ctx *c) {
    size_t nn = c->nn;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < (long)nn; i++) {
        if (c->solid[i]) {
            for (int q = 0; q < 18; q++) c->fpost[q * nn + i] = 0.0;
            continue;
        }
        double f[9], fp[9], oR[9], oB[9];
        for (int a = 0; a < 9; a++)
            f[a] = c->f[(0 * 9 + a) * nn + i] + c->f[(1 * 9 + a) * nn + i]; /* Sec. II A */
        double rho = c->rhoR[i] + c->rhoB[i];
        collide_node(&c->p, c->Minv, f, rho, c->ux[i], c->uy[i], c->Fx[i], c->Fy[i],
                     c->rhoN[i], fp);
        orc_recolor(fp, c->rhoR[i], c->rhoB[i], c->nvx[i], c->nvy[i], c->p.beta, oR, oB);
        for (int a = 0; a < 9; a++) {
            c->fpost[(0 * 9 + a) * nn + i] = oR[a];
            c->fpost[(1 * 9 + a) * nn + i] = oB[a];
        }
    }
}

/* Eq. 15 with half-way bounce-back, then open-boundary completion. */
static void pass_stream(orc_ctx *c) {
    size_t nn = c->nn;
    int nx = c->nx;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < c->ny; y++)
        for (int x = 0; x < nx; x++) {
            size_t i = (size_t)y * nx + x;
            if (c->solid[i]) {
                for (int q = 0; q < 18; q++) c->fn[q * nn + i] = 0.0;
                continue;
            }
            for (int a = 0; a < 9; a++) {
                int xs = x - EX[a], ys = wrap_y(c, y - EY[a]);
                if (c->p.open_x && (xs < 0 || xs >= nx)) {
                    c->fn[(0 * 9 + a) * nn + i] = 0.0; /* filled by the completion below */
                    c->fn[(1 * 9 + a) * nn + i] = 0.0;
                    continue;
                }
                xs = ((xs % nx) + nx) % nx;
                size_t s = (size_t)ys * nx + xs;
                for (int k = 0; k < 2; k++) {
                    if (c->solid[s]) /* half-way bounce-back */
                        c->fn[(k * 9 + a) * nn + i] = c->fpost[(k * 9 + OPP[a]) * nn + i];
                    else
                        c->fn[(k * 9 + a) * nn + i] = c->fpost[(k * 9 + a) * nn + s];
                }
            }
        }
    if (!c->p.open_x) return;

    /* Zou-He velocity inlet at x = 0: unknowns 1, 5, 8 of the total f, injected red. */
    for (int y = 0; y < c->ny; y++) {
        size_t i = (size_t)y * nx;
        if (c->solid[i]) continue;
        double t[9];
        for (int a = 0; a < 9; a++) t[a] = c->fn[a * nn + i] + c->fn[(9 + a) * nn + i];
        double u = c->inlet_ux[y];
        double rho = (t[0] + t[2] + t[4] + 2.0 * (t[3] + t[6] + t[7])) / (1.0 - u);
        double f1 = t[3] + (2.0 / 3.0) * rho * u;
        double f5 = t[7] - 0.5 * (t[2] - t[4]) + (1.0 / 6.0) * rho * u;
        double f8 = t[6] + 0.5 * (t[2] - t[4]) + (1.0 / 6.0) * rho * u;
        c->fn[1 * nn + i] = f1;
        c->fn[5 * nn + i] = f5;
        c->fn[8 * nn + i] = f8;
        c->fn[(9 + 1) * nn + i] = 0.0;
        c->fn[(9 + 5) * nn + i] = 0.0;
        c->fn[(9 + 8) * nn + i] = 0.0;
    }
    /* Convective outlet at x = nx-1 for the unknowns 3, 6, 7. */
    static const int UNK[3] = {3, 6, 7};
    double U = c->p.outlet_u;
    for (int y = 0; y < c->ny; y++) {
        size_t i = (size_t)y * nx + (nx - 1);
        if (c->solid[i]) continue;
        size_t im = i - 1;
        double cr = c->rhoR[i] / (c->rhoR[i] + c->rhoB[i]);
        double cb = c->rhoB[i] / (c->rhoR[i] + c->rhoB[i]);
        for (int q = 0; q < 3; q++) {
            int a = UNK[q];
            double old = c->f[a * nn + i] + c->f[(9 + a) * nn + i];
            double val;
            if (c->solid[im]) {
                val = old;
            } else {
                double inner = c->fn[a * nn + im] + c->fn[(9 + a) * nn + im];
                val = (old + U * inner) / (1.0 + U);
            }
            c->fn[a * nn + i] = cr * val;
            c->fn[(9 + a) * nn + i] = cb * val;
        }
    }
}

void orc_step(orc_ctx *c, int nsteps) {
    for (int s = 0; s < nsteps; s++) {
        prepare(c);
        pass_collide(c);
        pass_stream(c);
        double *t = c->f;
        c->f = c->fn;
        c->fn = t;
        c->step++;
    }
}

/* ------------------------------------------------------------ accessors */

void orc_get_pops(const orc_ctx *c, double *out) { memcpy(out, c->f, 18 * c->nn * sizeof(double)); }
void orc_set_pops(orc_ctx *c, const double *in) { memcpy(c->f, in, 18 * c->nn * sizeof(double)); }
long long orc_step_count(const orc_ctx *c) { return c->step; }

/* Recompute the pre-collision fields of the current populations and copy one out:
 * 0 rhoR, 1 rhoB, 2 rhoN (virtual values on outermost solid nodes), 3 gx, 4 gy
 * (corrected), 5 nx, 6 ny (virtual on solid), 7 kappa, 8 Fx, 9 Fy, 10 ux, 11 uy. */
int orc_fields(orc_ctx *c, int which, double *out) {
    double *src[12] = {c->rhoR, c->rhoB, c->rhoN, c->gx, c->gy, c->nvx,
                       c->nvy, c->kap, c->Fx, c->Fy, c->ux, c->uy};
    if (which < 0 || which > 11) return -1;
    prepare(c);
    memcpy(out, src[which], c->nn * sizeof(double));
    return 0;
}

void orc_classes(const orc_ctx *c, uint8_t *out) { memcpy(out, c->cls, c->nn); }
void orc_wall_normals(const orc_ctx *c, double *out) { memcpy(out, c->ns, 2 * c->nn * sizeof(double)); }

/* Per-colour mass over fluid nodes, serial and in a fixed order. */
void orc_mass(const orc_ctx *c, double *out) {
    double mR = 0.0, mB = 0.0;
    for (size_t i = 0; i < c->nn; i++) {
        if (c->solid[i]) continue;
        for (int a = 0; a < 9; a++) {
            mR += c->f[a * c->nn + i];
            mB += c->f[(9 + a) * c->nn + i];
        }
    }
    out[0] = mR;
    out[1] = mB;
}

void orc_matrices(double *M, double *Minv) {
    memcpy(M, MROW, sizeof(MROW));
    invert9(MROW, Minv);
}

void orc_lattice(int *ex, int *ey, double *w) {
    for (int a = 0; a < 9; a++) {
        ex[a] = EX[a];
        ey[a] = EY[a];
        w[a] = W[a];
    }
}

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
