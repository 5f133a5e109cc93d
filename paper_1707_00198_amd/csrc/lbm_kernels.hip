// Device code of lbmcg: one fused kernel per time step of the two-colour D2Q9 lattice
// Boltzmann method with the geometric wetting boundary (arXiv:1707.00198, Sec. II).
//
// Data layout (per context, all domains concatenated in every node plane):
//   populations: 9 direction planes of the storage type, holding deviations f - w rho0 of
//                the post-collision total distribution of each node (pull streaming);
//   colour state: c = rho_R / rho and v = beta (rho_R rho_B / rho) n of the node's last
//                collision, one plane each.  The recoloured per-colour populations of Eq. 14
//                are f''_{a,R} = c f'_a + w_a e_a . v and f''_{a,B} = (1 - c) f'_a - w_a e_a . v,
//                so the red population arriving at x along a is reconstructed at its
//                destination from the source node's (c, v) - an exact rewrite of Eqs. 14-16
//                that stores 12 values per node instead of 18.
//
// The step kernel marches a 64-column window (56 output columns plus a 4-column halo on each
// side) up a chunk of rows.  Every iteration advances four rows through five stages kept in
// LDS ring buffers, each lagging the previous one by a row:
//   A  pull the 9 populations (bounce-back, inlet and outlet completion), rho_R, rho_B, rho^N
//   B  virtual rho^N on outermost solid nodes (Eq. 29)
//   C  colour gradient (Eq. 28), wetting correction on outermost fluid nodes (Eqs. 30-36),
//      interface normal n (Eq. 22)
//   D  virtual normals on outermost solid nodes (Eq. 29, second boundary condition)
//   E  curvature (Eq. 13), CSF force (Eq. 10), velocity (Eq. 17), local viscosity (Eqs. 18,
//      5), MRT collision with Guo forcing (Eqs. 1-9), recolouring state (Eq. 14), store.
// Stage E of a row runs on the same thread that did stage A of that row one iteration
// earlier, so the populations stay in registers: each population is read once from HBM and
// written once per step (halo columns are re-read by the neighbouring window, from cache).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lbm_internal.h"

namespace lbmcg {

// D2Q9 velocity set in the paper's numbering.
__device__ constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

template <class AT>
__device__ __forceinline__ AT wgt(int a) {
    return a == 0 ? AT(4.0 / 9.0) : (a < 5 ? AT(1.0 / 9.0) : AT(1.0 / 36.0));
}

// ------------------------------------------------------------------ storage codec
template <class T>
struct Codec;
template <>
struct Codec<double> {
    using AT = double;
    __device__ static double load(const double *p, float) { return *p; }
    __device__ static void store(double *p, double v, float) { *p = v; }
};
template <>
struct Codec<float> {
    using AT = float;
    __device__ static float load(const float *p, float) { return *p; }
    __device__ static void store(float *p, float v, float) { *p = v; }
};
template <>
struct Codec<__half> {
    using AT = float;
    __device__ static float load(const __half *p, float inv_scale) {
        return __half2float(*p) * inv_scale;
    }
    __device__ static void store(__half *p, float v, float scale) {
        *p = __float2half_rn(v * scale);
    }
};

__device__ __forceinline__ int wrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

__device__ __forceinline__ size_t node_at(const DomDev &D, int x, int y) {
    return (size_t)D.off + (size_t)y * D.nx + x;
}

// Deviation of the post-streaming total population of direction a at node (x, y), for the
// interior pull: from the source node, or by half-way bounce-back from the node itself.
template <class T, class AT>
__device__ __forceinline__ AT pull_total(const StepArgs<T, AT> &A, const DomDev &D, int x, int y,
                                         uint32_t m, int a) {
    if (m & (1u << (OPP[a] - 1))) {
        return Codec<T>::load(A.fin + OPP[a] * A.plane + node_at(D, x, y), D.inv_scale[OPP[a]]);
    }
    int xs = x - EX[a], ys = wrap(y - EY[a], D.ny);
    if (!D.open_x) xs = wrap(xs, D.nx);
    return Codec<T>::load(A.fin + a * A.plane + node_at(D, xs, ys), D.inv_scale[a]);
}

// Post-streaming populations of fluid node (x, y) as deviations d[a], with the colour state
// (cs, vs) of the collision each one comes from.  Completes inlet (Zou-He, red) and outlet
// (convective) unknowns; with write_hist the completed outlet values are kept for the next
// step.
template <class T, class AT>
__device__ __forceinline__ void gather(const StepArgs<T, AT> &A, const DomDev &D, int x, int y,
                                       uint32_t m, bool write_hist, AT d[9], AT cs[9], AT vsx[9],
                                       AT vsy[9]) {
    const size_t self = node_at(D, x, y);
    if (A.own) {
        const AT c = A.cin[self];
#pragma unroll
        for (int a = 0; a < 9; a++) {
            d[a] = Codec<T>::load(A.fin + a * A.plane + self, D.inv_scale[a]);
            cs[a] = c;
            vsx[a] = AT(0);
            vsy[a] = AT(0);
        }
    } else {
        const AT cself = A.cin[self], vxs = A.vxin[self], vys = A.vyin[self];
#pragma unroll
        for (int a = 0; a < 9; a++) {
            if (a == 0) {
                d[0] = Codec<T>::load(A.fin + self, D.inv_scale[0]);
                cs[0] = cself;
                vsx[0] = AT(0);
                vsy[0] = AT(0);
                continue;
            }
            int xs = x - EX[a];
            const bool outside = D.open_x && (xs < 0 || xs >= D.nx);
            if (outside) {  // completed below
                d[a] = AT(0);
                cs[a] = cself;
                vsx[a] = AT(0);
                vsy[a] = AT(0);
            } else if (m & (1u << (OPP[a] - 1))) {  // half-way bounce-back
                d[a] = Codec<T>::load(A.fin + OPP[a] * A.plane + self, D.inv_scale[OPP[a]]);
                cs[a] = cself;
                vsx[a] = -vxs;
                vsy[a] = -vys;
            } else {
                if (!D.open_x) xs = wrap(xs, D.nx);
                const size_t s = node_at(D, xs, wrap(y - EY[a], D.ny));
                d[a] = Codec<T>::load(A.fin + a * A.plane + s, D.inv_scale[a]);
                cs[a] = A.cin[s];
                vsx[a] = A.vxin[s];
                vsy[a] = A.vyin[s];
            }
        }
        if (D.open_x && x == 0) {
            // Zou-He velocity inlet on the total f; injected fluid is pure red.
            const AT u = A.inlet[D.io_off + y];
            const AT rho = (AT(D.rho0) + d[0] + d[2] + d[4] + AT(2) * (d[3] + d[6] + d[7])) /
                           (AT(1) - u);
            const AT ru = rho * u;
            d[1] = d[3] + AT(2.0 / 3.0) * ru;
            d[5] = d[7] - AT(0.5) * (d[2] - d[4]) + AT(1.0 / 6.0) * ru;
            d[8] = d[6] + AT(0.5) * (d[2] - d[4]) + AT(1.0 / 6.0) * ru;
            cs[1] = cs[5] = cs[8] = AT(1);
        }
        if (D.open_x && x == D.nx - 1) {
            // Convective outlet f_a <- [f_a(t) + U f_a(x - 1, t + 1)] / (1 + U), coloured
            // with this node's red fraction.
            const AT U = AT(D.outlet_u);
            const size_t im = self - 1;
            const uint32_t mm = A.mask[im];
            const AT *h = A.hist_in + (D.io_off + y) * 3;
            const int unk[3] = {3, 6, 7};
#pragma unroll
            for (int q = 0; q < 3; q++) {
                const int a = unk[q];
                AT v = h[q];
                if (!(mm & SELF_SOLID)) v = (v + U * pull_total(A, D, x - 1, y, mm, a)) / (AT(1) + U);
                d[a] = v;
            }
        }
    }
    if (write_hist && D.open_x && x == D.nx - 1) {
        AT *h = A.hist_out + (D.io_off + y) * 3;
        h[0] = d[3];
        h[1] = d[6];
        h[2] = d[7];
    }
}

// Contact-angle correction of the colour gradient on an outermost fluid node (Eqs. 30-36):
// keep |grad rho^N|, replace its direction by the wall normal rotated by +theta or -theta,
// whichever is closer to the estimated direction (ties pick +theta).  Evaluated without
// contraction so that the selection rounds like a plain IEEE evaluation of the same formulas.
template <class AT>
__device__ __forceinline__ void wetting_correct(AT nsx, AT nsy, AT ct, AT st, AT eps, AT &gx,
                                                AT &gy) {
#pragma clang fp contract(off)
    const AT g = sqrt(gx * gx + gy * gy);
    if (!(g > eps)) return;
    const AT ex = gx / g, ey = gy / g;
    const AT n1x = nsx * ct - nsy * st, n1y = nsx * st + nsy * ct;
    const AT n2x = nsx * ct + nsy * st, n2y = -nsx * st + nsy * ct;
    const AT d1 = sqrt((n1x - ex) * (n1x - ex) + (n1y - ey) * (n1y - ey));
    const AT d2 = sqrt((n2x - ex) * (n2x - ex) + (n2y - ey) * (n2y - ey));
    if (d1 <= d2) {
        gx = g * n1x;
        gy = g * n1y;
    } else {
        gx = g * n2x;
        gy = g * n2y;
    }
}

// Red and blue densities (Eq. 16) of the gathered populations.
template <class AT>
__device__ __forceinline__ void colour_densities(const AT d[9], const AT cs[9], const AT vsx[9],
                                                 const AT vsy[9], AT rho0, AT &rR, AT &rB) {
    rR = AT(0);
    rB = AT(0);
#pragma unroll
    for (int a = 0; a < 9; a++) {
        const AT fa = wgt<AT>(a) * rho0 + d[a];
        const AT t = wgt<AT>(a) * (AT(EX[a]) * vsx[a] + AT(EY[a]) * vsy[a]);
        rR += cs[a] * fa + t;
        rB += (AT(1) - cs[a]) * fa - t;
    }
}

// --------------------------------------------------------------------- step kernel
template <class T>
__global__ __launch_bounds__(TILE_LANES *TILE_WAVES) void step_kernel(
    const StepArgs<T, typename Codec<T>::AT> A) {
    using AT = typename Codec<T>::AT;
    __shared__ AT s_rn[RING][TILE_LANES];
    __shared__ AT s_nx[RING][TILE_LANES], s_ny[RING][TILE_LANES];
    __shared__ AT s_gx[RING][TILE_LANES], s_gy[RING][TILE_LANES];
    __shared__ uint16_t s_m[RING][TILE_LANES];

    const WorkItem it = A.items[blockIdx.x];
    const DomDev &D = A.doms[it.dom];
    const int w = threadIdx.x / TILE_LANES;
    const int lane = threadIdx.x % TILE_LANES;
    const int base = it.x0 - HALO;
    const int X = base + lane;  // raw column of this lane
    int xe, lm, lp;             // node column, LDS lanes of the x-1 / x+1 stencil neighbours
    if (D.open_x) {
        xe = min(max(X, 0), D.nx - 1);
        lm = max(xe - 1, 0) - base;
        lp = min(xe + 1, D.nx - 1) - base;
    } else {
        xe = wrap(X, D.nx);
        lm = lane - 1;
        lp = lane + 1;
    }
    const int lanes_of[3] = {lm, lane, lp};
    const bool out_lane = lane >= HALO && lane < TILE_LANES - HALO && X < D.nx;

    const AT rho0 = AT(D.rho0);
    const AT eps = AT(D.eps);

    // Stage E of iteration r collides the row this thread gathered in stage A of iteration
    // r - 4; stage A of iteration r already gathers the next row, hence two register sets.
    AT d[9], dn[9];
    AT rR = AT(0), rB = AT(0), rN = AT(0), rRn = AT(0), rBn = AT(0), rNn = AT(0);
#pragma unroll
    for (int a = 0; a < 9; a++) d[a] = dn[a] = AT(0);

    const int y0 = it.y0, y1 = it.y1;
    for (int r = y0 - 2 * HALO; r < y1; r += TILE_WAVES) {
        // ---- A: gather, densities, colour indicator
        {
            const int ya = r + HALO + w;
            uint32_t m = SELF_SOLID;
            AT rn = AT(0);
            if (ya >= y0 - HALO && ya < y1 + HALO) {
                const int yw = wrap(ya, D.ny);
                m = A.mask[node_at(D, xe, yw)];
                if (!(m & SELF_SOLID)) {
                    AT cs[9], vsx[9], vsy[9];
                    gather(A, D, xe, yw, m, true, dn, cs, vsx, vsy);
                    colour_densities(dn, cs, vsx, vsy, rho0, rRn, rBn);
                    rn = (rRn - rBn) / (rRn + rBn);
                    rNn = rn;
                }
            }
            s_m[ya & (RING - 1)][lane] = (uint16_t)m;
            s_rn[ya & (RING - 1)][lane] = rn;
        }
        __syncthreads();
        // ---- B: virtual colour indicator on outermost solid nodes
        {
            const int yb = r + HALO - 1 + w;
            const int sl = yb & (RING - 1);
            if (lane >= 1 && lane < TILE_LANES - 1 && yb >= y0 - HALO + 1 && yb < y1 + HALO - 1) {
                const uint32_t m = s_m[sl][lane];
                if (m & SOLID_BND) {
                    AT num = AT(0), den = AT(0);
#pragma unroll
                    for (int a = 1; a < 9; a++) {
                        if (m & (1u << (a - 1))) continue;
                        const AT wa = wgt<AT>(a);
                        num += wa * s_rn[(yb + EY[a]) & (RING - 1)][lanes_of[EX[a] + 1]];
                        den += wa;
                    }
                    s_rn[sl][lane] = num / den;
                }
            }
        }
        __syncthreads();
        // ---- C: colour gradient, wetting correction, interface normal
        {
            const int yc = r + HALO - 2 + w;
            const int sl = yc & (RING - 1);
            if (lane >= 2 && lane < TILE_LANES - 2 && yc >= y0 - HALO + 2 && yc < y1 + HALO - 2) {
                const uint32_t m = s_m[sl][lane];
                AT gx = AT(0), gy = AT(0), nx = AT(0), ny = AT(0);
                if (!(m & SELF_SOLID)) {
#pragma clang fp contract(off)
                    AT sx = AT(0), sy = AT(0);
#pragma unroll
                    for (int a = 1; a < 9; a++) {
                        const AT v = s_rn[(yc + EY[a]) & (RING - 1)][lanes_of[EX[a] + 1]];
                        if (EX[a]) sx += wgt<AT>(a) * v * AT(EX[a]);
                        if (EY[a]) sy += wgt<AT>(a) * v * AT(EY[a]);
                    }
                    gx = AT(3) * sx;
                    gy = AT(3) * sy;
                    if (m & FLUID_BND) {
                        const size_t nd = node_at(D, xe, wrap(yc, D.ny));
                        wetting_correct(A.nsx[nd], A.nsy[nd], AT(D.cos_t), AT(D.sin_t), eps, gx, gy);
                    }
                    const AT g = sqrt(gx * gx + gy * gy);
                    if (g > eps) {
                        nx = gx / g;
                        ny = gy / g;
                    }
                }
                s_gx[sl][lane] = gx;
                s_gy[sl][lane] = gy;
                s_nx[sl][lane] = nx;
                s_ny[sl][lane] = ny;
            }
        }
        __syncthreads();
        // ---- D: virtual interface normals on outermost solid nodes
        {
            const int yd = r + HALO - 3 + w;
            const int sl = yd & (RING - 1);
            if (lane >= 3 && lane < TILE_LANES - 3 && yd >= y0 - 1 && yd < y1 + 1) {
                const uint32_t m = s_m[sl][lane];
                if (m & SOLID_BND) {
                    AT numx = AT(0), numy = AT(0), den = AT(0);
#pragma unroll
                    for (int a = 1; a < 9; a++) {
                        if (m & (1u << (a - 1))) continue;
                        const AT wa = wgt<AT>(a);
                        const int s2 = (yd + EY[a]) & (RING - 1);
                        const int l2 = lanes_of[EX[a] + 1];
                        numx += wa * s_nx[s2][l2];
                        numy += wa * s_ny[s2][l2];
                        den += wa;
                    }
                    s_nx[sl][lane] = numx / den;
                    s_ny[sl][lane] = numy / den;
                }
            }
        }
        __syncthreads();
        // ---- E: curvature, force, collision, recolouring state, store
        {
            const int ye = r + w;
            const int sl = ye & (RING - 1);
            if (out_lane && ye >= y0 && ye < y1 && !(s_m[sl][lane] & SELF_SOLID)) {
                AT dxnx = AT(0), dynx = AT(0), dxny = AT(0), dyny = AT(0);
                {
#pragma clang fp contract(off)
#pragma unroll
                for (int a = 1; a < 9; a++) {
                    const int s2 = (ye + EY[a]) & (RING - 1);
                    const int l2 = lanes_of[EX[a] + 1];
                    const AT vx = s_nx[s2][l2], vy = s_ny[s2][l2];
                    if (EX[a]) {
                        dxnx += wgt<AT>(a) * vx * AT(EX[a]);
                        dxny += wgt<AT>(a) * vy * AT(EX[a]);
                    }
                    if (EY[a]) {
                        dynx += wgt<AT>(a) * vx * AT(EY[a]);
                        dyny += wgt<AT>(a) * vy * AT(EY[a]);
                    }
                }
                dxnx *= AT(3);
                dynx *= AT(3);
                dxny *= AT(3);
                dyny *= AT(3);
                }
                const AT nx = s_nx[sl][lane], ny = s_ny[sl][lane];
                const AT gx = s_gx[sl][lane], gy = s_gy[sl][lane];
                const AT kappa = -nx * nx * dyny - ny * ny * dxnx + nx * ny * (dynx + dxny);
                const AT Fx = AT(D.half_sigma) * kappa * gx;
                const AT Fy = AT(D.half_sigma) * kappa * gy;

                // moments of the deviations
                const AT drho = d[0] + d[1] + d[2] + d[3] + d[4] + d[5] + d[6] + d[7] + d[8];
                const AT sa = d[1] + d[2] + d[3] + d[4];
                const AT sd = d[5] + d[6] + d[7] + d[8];
                const AT jx = d[1] - d[3] + d[5] - d[6] - d[7] + d[8];
                const AT jy = d[2] - d[4] + d[5] + d[6] - d[7] - d[8];
                const AT m1 = AT(-4) * d[0] - sa + AT(2) * sd;
                const AT m2 = AT(4) * d[0] - AT(2) * sa + sd;
                const AT m4 = AT(-2) * (d[1] - d[3]) + (d[5] - d[6] - d[7] + d[8]);
                const AT m6 = AT(-2) * (d[2] - d[4]) + (d[5] + d[6] - d[7] - d[8]);
                const AT m7 = d[1] - d[2] + d[3] - d[4];
                const AT m8 = d[5] - d[6] + d[7] - d[8];

                const AT rho = rho0 + drho;
                const AT ux = (jx + AT(0.5) * Fx) / rho;
                const AT uy = (jy + AT(0.5) * Fy) / rho;
                const AT inv_nu = (AT(1) + rN) * AT(D.inv2nu_r) + (AT(1) - rN) * AT(D.inv2nu_b);
                const AT nu = AT(1) / inv_nu;
                const AT sv = AT(1) / (AT(3) * nu + AT(0.5));
                const AT se = AT(D.s_e), seps = AT(D.s_eps), sq = AT(D.s_q);

                const AT uu = ux * ux + uy * uy;
                const AT r3uu = AT(3) * rho * uu;
                const AT uF = ux * Fx + uy * Fy;
                // post-collision moments of the deviations (Eqs. 1, 2, 8 in moment space)
                const AT p0 = drho;
                const AT p1 = m1 - se * (m1 + AT(2) * drho - r3uu) + (AT(1) - AT(0.5) * se) * (AT(6) * uF);
                const AT p2 = m2 - seps * (m2 - drho + r3uu) - (AT(1) - AT(0.5) * seps) * (AT(6) * uF);
                const AT p3 = rho * ux + AT(0.5) * Fx;
                const AT p4 = m4 - sq * (m4 + rho * ux) - (AT(1) - AT(0.5) * sq) * Fx;
                const AT p5 = rho * uy + AT(0.5) * Fy;
                const AT p6 = m6 - sq * (m6 + rho * uy) - (AT(1) - AT(0.5) * sq) * Fy;
                const AT p7 = m7 - sv * (m7 - rho * (ux * ux - uy * uy)) +
                              (AT(1) - AT(0.5) * sv) * (AT(2) * (ux * Fx - uy * Fy));
                const AT p8 = m8 - sv * (m8 - rho * ux * uy) + (AT(1) - AT(0.5) * sv) * (ux * Fy + uy * Fx);
                // back to populations: M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
                const AT a0 = p0 * AT(1.0 / 9.0), a1 = p1 * AT(1.0 / 36.0), a2 = p2 * AT(1.0 / 36.0);
                const AT a3 = p3 * AT(1.0 / 6.0), a4 = p4 * AT(1.0 / 12.0);
                const AT a5 = p5 * AT(1.0 / 6.0), a6 = p6 * AT(1.0 / 12.0);
                const AT a7 = p7 * AT(0.25), a8 = p8 * AT(0.25);
                AT o[9];
                o[0] = a0 - AT(4) * a1 + AT(4) * a2;
                const AT ax = a0 - a1 - AT(2) * a2;
                o[1] = ax + a3 - AT(2) * a4 + a7;
                o[2] = ax + a5 - AT(2) * a6 - a7;
                o[3] = ax - a3 + AT(2) * a4 + a7;
                o[4] = ax - a5 + AT(2) * a6 - a7;
                const AT ad = a0 + AT(2) * a1 + a2;
                o[5] = ad + a3 + a4 + a5 + a6 + a8;
                o[6] = ad - a3 - a4 + a5 + a6 - a8;
                o[7] = ad - a3 - a4 - a5 - a6 + a8;
                o[8] = ad + a3 + a4 - a5 - a6 - a8;

                // recolouring state (Eq. 14)
                const AT rs = rR + rB;
                const AT c = rR / rs;
                const AT b = AT(D.beta) * (rR * rB / rs);
                const size_t nd = node_at(D, xe, wrap(ye, D.ny));
#pragma unroll
                for (int a = 0; a < 9; a++) Codec<T>::store(A.fout + a * A.plane + nd, o[a], D.scale[a]);
                A.cout[nd] = c;
                A.vxout[nd] = b * nx;
                A.vyout[nd] = b * ny;
                if (!(isfinite(rho) && isfinite(ux) && isfinite(uy))) atomicOr(A.flag, 1);
            }
        }
#pragma unroll
        for (int a = 0; a < 9; a++) d[a] = dn[a];
        rR = rRn;
        rB = rBn;
        rN = rNn;
        // No barrier here: the next stage A writes ring rows r + 8 .. r + 11 of s_rn / s_m,
        // which alias rows r .. r + 3.  Of those, stage E reads only s_m of its own row, which
        // only its own wavefront rewrites; the n and g rings are not touched by stage A.
    }
}

// ------------------------------------------------------------- decode to FP64 fields
template <class T>
__global__ void read_kernel(const StepArgs<T, typename Codec<T>::AT> A, int dom, uint32_t which,
                            double *out) {
    using AT = typename Codec<T>::AT;
    const DomDev &D = A.doms[dom];
    const size_t nn = (size_t)D.nx * D.ny;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nn;
         i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % D.nx), y = (int)(i / D.nx);
        const uint32_t m = A.mask[D.off + i];
        double fR[9], fB[9], rR = 0.0, rB = 0.0;
        if (!(m & SELF_SOLID)) {
            AT d[9], cs[9], vsx[9], vsy[9];
            gather(A, D, x, y, m, false, d, cs, vsx, vsy);
#pragma unroll
            for (int a = 0; a < 9; a++) {
                const double fa = wgt<double>(a) * D.rho0 + (double)d[a];
                const double t = wgt<double>(a) * (EX[a] * (double)vsx[a] + EY[a] * (double)vsy[a]);
                fR[a] = (double)cs[a] * fa + t;
                fB[a] = (1.0 - (double)cs[a]) * fa - t;
                rR += fR[a];
                rB += fB[a];
            }
        } else {
#pragma unroll
            for (int a = 0; a < 9; a++) fR[a] = fB[a] = 0.0;
        }
        size_t p = 0;
        if (which & 1u) out[(p++) * nn + i] = rR;
        if (which & 2u) out[(p++) * nn + i] = rB;
        if (which & 4u) {
#pragma unroll
            for (int a = 0; a < 9; a++) out[(p + a) * nn + i] = fR[a];
#pragma unroll
            for (int a = 0; a < 9; a++) out[(p + 9 + a) * nn + i] = fB[a];
        }
    }
}

// ------------------------------------------------------- FP64 per-domain mass sums
constexpr int MASS_THREADS = 256;

template <class T>
__global__ __launch_bounds__(MASS_THREADS) void mass_partial_kernel(
    const StepArgs<T, typename Codec<T>::AT> A, int blocks_per_dom, double *partials) {
    using AT = typename Codec<T>::AT;
    const int dom = blockIdx.x / blocks_per_dom;
    const int b = blockIdx.x % blocks_per_dom;
    const DomDev &D = A.doms[dom];
    const size_t nn = (size_t)D.nx * D.ny;
    double sR = 0.0, sB = 0.0;
    for (size_t i = (size_t)b * MASS_THREADS + threadIdx.x; i < nn;
         i += (size_t)blocks_per_dom * MASS_THREADS) {
        const uint32_t m = A.mask[D.off + i];
        if (m & SELF_SOLID) continue;
        AT d[9], cs[9], vsx[9], vsy[9];
        gather(A, D, (int)(i % D.nx), (int)(i / D.nx), m, false, d, cs, vsx, vsy);
        for (int a = 0; a < 9; a++) {
            const double fa = wgt<double>(a) * D.rho0 + (double)d[a];
            const double t = wgt<double>(a) * (EX[a] * (double)vsx[a] + EY[a] * (double)vsy[a]);
            sR += (double)cs[a] * fa + t;
            sB += (1.0 - (double)cs[a]) * fa - t;
        }
    }
    __shared__ double shR[MASS_THREADS], shB[MASS_THREADS];
    shR[threadIdx.x] = sR;
    shB[threadIdx.x] = sB;
    __syncthreads();
    for (int s = MASS_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            shR[threadIdx.x] += shR[threadIdx.x + s];
            shB[threadIdx.x] += shB[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = shR[0];
        partials[2 * blockIdx.x + 1] = shB[0];
    }
}

__global__ void mass_final_kernel(const double *partials, int n_doms, int blocks_per_dom,
                                  double *out) {
    const int dom = blockIdx.x * blockDim.x + threadIdx.x;
    if (dom >= n_doms) return;
    double sR = 0.0, sB = 0.0;
    for (int b = 0; b < blocks_per_dom; b++) {
        sR += partials[2 * (dom * blocks_per_dom + b)];
        sB += partials[2 * (dom * blocks_per_dom + b) + 1];
    }
    out[2 * dom] = sR;
    out[2 * dom + 1] = sB;
}

// ------------------------------------------------------------------- launchers
template <class T>
static hipError_t step_t(const void *args, int n_items, hipStream_t s) {
    const auto &A = *static_cast<const StepArgs<T, typename Codec<T>::AT> *>(args);
    hipLaunchKernelGGL(step_kernel<T>, dim3(n_items), dim3(TILE_LANES * TILE_WAVES), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_step(int storage, const void *args, int n_items, int, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    switch (storage) {
        case 0: return step_t<double>(args, n_items, s);
        case 1: return step_t<float>(args, n_items, s);
        case 2: return step_t<__half>(args, n_items, s);
    }
    return hipErrorInvalidValue;
}

template <class T>
static hipError_t read_t(const void *args, int dom, int nx, int ny, uint32_t which, double *out,
                         hipStream_t s) {
    const auto &A = *static_cast<const StepArgs<T, typename Codec<T>::AT> *>(args);
    const size_t nn = (size_t)nx * ny;
    const int blocks = (int)((nn + 255) / 256 < 4096 ? (nn + 255) / 256 : 4096);
    hipLaunchKernelGGL(read_kernel<T>, dim3(blocks), dim3(256), 0, s, A, dom, which, out);
    return hipGetLastError();
}

hipError_t launch_read(int storage, const void *args, int dom, int nx, int ny, uint32_t which,
                       double *out, hipStream_t s) {
    switch (storage) {
        case 0: return read_t<double>(args, dom, nx, ny, which, out, s);
        case 1: return read_t<float>(args, dom, nx, ny, which, out, s);
        case 2: return read_t<__half>(args, dom, nx, ny, which, out, s);
    }
    return hipErrorInvalidValue;
}

template <class T>
static hipError_t mass_t(const void *args, int n_doms, double *partials, int bpd, double *out,
                         hipStream_t s) {
    const auto &A = *static_cast<const StepArgs<T, typename Codec<T>::AT> *>(args);
    hipLaunchKernelGGL(mass_partial_kernel<T>, dim3(n_doms * bpd), dim3(MASS_THREADS), 0, s, A,
                       bpd, partials);
    hipLaunchKernelGGL(mass_final_kernel, dim3((n_doms + 63) / 64), dim3(64), 0, s, partials,
                       n_doms, bpd, out);
    return hipGetLastError();
}

hipError_t launch_mass(int storage, const void *args, int n_doms, const int *, double *partials,
                       int bpd, double *out, hipStream_t s) {
    switch (storage) {
        case 0: return mass_t<double>(args, n_doms, partials, bpd, out, s);
        case 1: return mass_t<float>(args, n_doms, partials, bpd, out, s);
        case 2: return mass_t<__half>(args, n_doms, partials, bpd, out, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lbmcg
