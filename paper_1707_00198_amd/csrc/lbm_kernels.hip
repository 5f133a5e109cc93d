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
// The step kernel marches a 64-column window up a chunk of rows: 56 output columns and a
// 4-column halo on each side (the dependency radius next to walls), with the colour state of
// the column beyond each halo in two extra LDS columns; with FP64 arithmetic, 54 output columns
// and a 5-column halo whose outermost lanes hold that colour state.  Every iteration advances R rows (4 by default) through five stages kept
// in LDS ring buffers, each lagging the previous one by a row:
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
// Per-domain wetting variants of Sec. III A (scheme (b), Eq. 48; the surface-energy rule)
// change stages B-E.  A diagnostic launch runs the same kernel without writing the state and
// outputs the velocity of Eq. 17 and, optionally, the contact-line nodes instead.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <mutex>

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

// Reciprocal and square root: IEEE in FP64 (the FP64 path is checked element by element
// against a plain FP64 evaluation); the hardware's 1-ulp instructions in FP32.
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// a / b: IEEE in FP64; in FP32 the 1-ulp reciprocal refined by one Newton step, which removes
// the reciprocal's systematic bias (the red fraction c = rho_R / rho must not drift the
// colour masses).
__device__ __forceinline__ double quotient(double a, double b) { return a / b; }
__device__ __forceinline__ float quotient(float a, float b) {
    const float q = a * rcp(b);
    return fmaf(rcp(b), fmaf(-q, b, a), q);
}

// Colour indicator (Eq. 12), exactly +-1 in pure phases.
__device__ __forceinline__ double colour_indicator(double rR, double rB) { return (rR - rB) / (rR + rB); }
__device__ __forceinline__ float colour_indicator(float rR, float rB) {
    return rB == 0.0f ? 1.0f : (rR == 0.0f ? -1.0f : (rR - rB) * rcp(rR + rB));
}

// Unit interface normal (Eq. 22) from a gradient of modulus g > 0.
__device__ __forceinline__ void unit_normal(double gx, double gy, double g, double &nx, double &ny) {
    nx = gx / g;
    ny = gy / g;
}
__device__ __forceinline__ void unit_normal(float gx, float gy, float g, float &nx, float &ny) {
    const float ig = rcp(g);
    nx = gx * ig;
    ny = gy * ig;
}

// Accumulate s +/- w*v.  In FP64 the product is rounded before the sum (no contraction), as in
// a plain IEEE evaluation: the colour gradient feeds branches (|grad| > eps, the contact-angle
// selection) whose symmetric ties must round the same way.
__device__ __forceinline__ double acc_nc(double s, double w, double v, int sign) {
#pragma clang fp contract(off)
    const double t = w * v;
    return sign > 0 ? s + t : s - t;
}
__device__ __forceinline__ float acc_nc(float s, float w, float v, int sign) {
    return sign > 0 ? s + w * v : s - w * v;
}

// ------------------------------------------------------------------ storage codec
template <class T>
struct Codec;
template <>
struct Codec<double> {
    using AT = double;
    __device__ static double load(const double *p, int) { return *p; }
    __device__ static double decode(double v, int) { return v; }
    __device__ static double encode(double v, int) { return v; }
};
template <>
struct Codec<float> {
    using AT = float;
    __device__ static float load(const float *p, int) { return *p; }
    __device__ static float decode(float v, int) { return v; }
    __device__ static float encode(float v, int) { return v; }
};
template <>
struct Codec<__half> {
    using AT = float;
    // FP16 holds the deviation times 2^k(a), k = round(log2(256 / w_a)): 2^9, 2^11, 2^13 for
    // rest, axis and diagonal directions, which keeps typical deviations far from the FP16
    // subnormal range without risking overflow.
    __device__ static constexpr float scale(int a) { return a == 0 ? 512.0f : (a < 5 ? 2048.0f : 8192.0f); }
    __device__ static float load(const __half *p, int a) { return __half2float(*p) * (1.0f / scale(a)); }
    // one mixed-precision FMA (binary16 source, FP32 result); the product is exact
    __device__ static float decode(__half v, int a) { return __builtin_fmaf(__half2float(v), 1.0f / scale(a), 0.0f); }
    // The store path's rounding, stochastic as for the 11-bit-fraction format (Codec<C16>): a
    // uniform random 13-bit offset (bits 2a .. 2a + 12 of rnd) is added to the 13 bits of the
    // scaled FP32 value that binary16 drops, and the conversion truncates (v_cvt_pkrtz), so the
    // magnitude rounds up with a probability equal to the dropped fraction wherever binary16 is
    // normal (below 2^-14 the dropped part is wider and the rounding leans towards zero);
    // values beyond the largest finite half truncate to it.  The binary16 bits come back in the
    // lower half of the word.
    __device__ static uint32_t encode_sr(float v, int a, uint32_t rnd) {
        const uint32_t b = __float_as_uint(v * scale(a)) + __builtin_amdgcn_ubfe(rnd, 2 * a, 13);
        return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(__uint_as_float(b), 0.0f));
    }
};

template <>
struct Codec<C16> {
    using AT = float;
    // The 15 exponent-and-fraction bits, moved to bit 12 of an FP32 word, read as an FP32
    // number 2^(e - 127) (1 + f / 2^11) (or its subnormal for e = 0); one multiplication by
    // 2^(127 - 7) / scale(a) then gives the deviation.  FP32 subnormals are kept (the kernels
    // run with denormals enabled), so the small values decode exactly.
    __device__ static constexpr float dec(int a) {
        return a == 0 ? 0x1p111f : (a < 5 ? 0x1p109f : 0x1p107f);
    }
    __device__ static constexpr float enc(int a) {
        return a == 0 ? 0x1p-111f : (a < 5 ? 0x1p-109f : 0x1p-107f);
    }
    __device__ static float decode(C16 v, int a) {
        const uint32_t u = v.bits;
        return __uint_as_float(((u & 0x7FFFu) << 12) | ((u & 0x8000u) << 16)) * dec(a);
    }
    __device__ static float load(const C16 *p, int a) { return decode(*p, a); }
    // The store path's rounding: stochastic, so that rounding errors carry no systematic part
    // that could add up over many steps (with round-to-nearest the 16384 x 512 displacement
    // channel's finger tip ran 0.36 % fast over 30000 steps; with this rounding 0.02 %).  The
    // scaled value is clamped to the largest code while still an FP32 number (0x07FFF000 as
    // bits, so no carry can reach the unused exponent bits), then a uniform random 12-bit
    // offset is added to the 12 bits that the code drops: the magnitude rounds up with a
    // probability equal to the dropped fraction, and the sign is carried over.  The result is
    // one of the two codes next to the value (exact values stay exact), in the lower 16 bits of
    // the word (the upper bits undefined).  The offset is bits 2a .. 2a + 11 of rnd for
    // direction a (one bit-field extract, as round-to-nearest needs one for its tie bit).
    __device__ static uint32_t encode_sr(float v, int a, uint32_t rnd) {
        constexpr float top = 0x1.fffp-112f;  // bits 0x07FFF000
        const float x = __builtin_amdgcn_fmed3f(v * enc(a), -top, top);
        const uint32_t t = __float_as_uint(x) + __builtin_amdgcn_ubfe(rnd, 2 * a, 12);
        return (t >> 12) | ((t >> 16) & 0x8000u);
    }
};

// Random bits for the stochastic rounding of one node's stores in either 16-bit format: a hash
// of the node's byte offset within its domain and of the bit pattern of its post-collision rest
// population, so the bits differ from node to node and from step to step, and a domain's
// results do not depend on the tile shape or on the other domains of its batch.  Two rounds of
// xor-shift and a 24-bit multiply (full-rate v_mul_u32_u24, where a 32-bit multiply issues at
// a quarter of the rate); the xor-shift before each multiply folds the upper bits in.
__device__ __forceinline__ uint32_t round_bits(uint32_t node_bytes, float v) {
    uint32_t x = node_bytes ^ __float_as_uint(v);
    x ^= x >> 16;
    uint32_t h = __umul24(x, 0x9E3779u);
    h ^= h >> 13;
    h = __umul24(h, 0x85EBCAu);
    return h ^ (h >> 16);
}

// Periodic wrap of an index that is usually already in [0, n): one compare on the fast path.
// Element access into one node plane: a uniform base pointer plus a 32-bit byte offset, so
// that each access needs one vector offset (planes are below 2^31 bytes, checked on the host).
template <class V>
struct Plane {
    V *p;
    __device__ __forceinline__ Plane(const V *b, uint32_t) : p(const_cast<V *>(b)) {}
    __device__ __forceinline__ V load(uint32_t i) const {
        return *reinterpret_cast<const V *>(reinterpret_cast<const char *>(p) + i * (uint32_t)sizeof(V));
    }
    __device__ __forceinline__ void store(uint32_t i, V v) const {
        *reinterpret_cast<V *>(reinterpret_cast<char *>(p) + i * (uint32_t)sizeof(V)) = v;
    }
};

// Domain parameters are read through the constant address space: every read is wave-uniform,
// so it becomes a scalar load, and a reload after vector stores never waits for the vector
// loads in flight.
using DomC = const __attribute__((address_space(4))) DomDev;
template <class AT>
using ParC = const __attribute__((address_space(4))) DomPar<AT>;
// parameters of a domain in the arithmetic type AT
__device__ __forceinline__ ParC<double> &par(DomC &D, double) { return D.d; }
__device__ __forceinline__ ParC<float> &par(DomC &D, float) { return D.f; }

__device__ __forceinline__ int wrap(int v, int n) {
    if ((unsigned)v < (unsigned)n) return v;
    v %= n;
    return v < 0 ? v + n : v;
}

// Neighbourhood of node (x, y) of a domain: node offsets of the rows y-1, y, y+1 (periodic) and
// the columns x-1, x, x+1 (periodic, or clamped at an open x axis, where lo / hi flag that the
// column lies beyond the inlet / outlet).
struct Nbr {
    size_t row[3];
    int col[3];
    bool lo, hi;
};

__device__ __forceinline__ Nbr make_nbr(DomC &D, int x, int y) {
    Nbr n;
    const int ym = y == 0 ? D.ny - 1 : y - 1;
    const int yp = y == D.ny - 1 ? 0 : y + 1;
    n.row[0] = (size_t)D.off + (size_t)ym * D.nx;
    n.row[1] = (size_t)D.off + (size_t)y * D.nx;
    n.row[2] = (size_t)D.off + (size_t)yp * D.nx;
    n.col[1] = x;
    if (D.open_x) {
        n.lo = x == 0;
        n.hi = x == D.nx - 1;
        n.col[0] = n.lo ? x : x - 1;
        n.col[2] = n.hi ? x : x + 1;
    } else {
        n.lo = n.hi = false;
        n.col[0] = x == 0 ? D.nx - 1 : x - 1;
        n.col[2] = x == D.nx - 1 ? 0 : x + 1;
    }
    return n;
}

// Node the pull of direction a reads from: x - e_a.
__device__ __forceinline__ size_t pull_src(const Nbr &n, int a) {
    return n.row[1 - EY[a]] + n.col[1 - EX[a]];
}

// The pull of direction a crosses the inlet (x = 0, e_x = +1) or the outlet (x = nx-1, e_x = -1).
__device__ __forceinline__ bool pull_outside(const Nbr &n, int a) {
    return (n.lo && EX[a] == 1) || (n.hi && EX[a] == -1);
}

// Completes the post-streaming populations d[] of fluid node (x, y) whose interior pulls are
// already in d[] (and whose own-node snapshot values are in d[] in snapshot mode): half-way
// bounce-back on links from solid nodes, Zou-He inlet and convective outlet unknowns; and
// returns the red and blue densities of Eq. 16.  colour(a, c, vx, vy) yields the colour state
// of the pull source of direction a (a = 0: the node itself).
// BOUNCED: d[] already holds the bounced populations f_opp(a) of the node itself for pulls from
// solid nodes (the step kernel's prefetch redirects those loads).
template <bool BOUNCED, class T, class AT, class ColourFn>
__device__ __forceinline__ void finish_gather(const StepArgs<T, AT> &A, DomC &D, int x, int y,
                                              uint32_t m, const Nbr &nb, bool write_hist, AT d[9],
                                              AT &rR, AT &rB, ColourFn colour) {
    const size_t self = nb.row[1] + x;
    ParC<AT> &P = par(D, AT());
    const AT rho0 = P.rho0;
    AT cself, vxs, vys;
    colour(0, cself, vxs, vys);
    rR = AT(0);
    rB = AT(0);
    if (A.own) {
        // node-local snapshot: every population carries the node's own red fraction
        AT tot = AT(0);
#pragma unroll
        for (int a = 0; a < 9; a++) tot += wgt<AT>(a) * rho0 + d[a];
        rR = cself * tot;
        rB = tot - rR;
    } else if ((m & 0xFFu) == 0u && !nb.lo && !nb.hi) {
        // interior node: every population is pulled from a fluid neighbour
        AT tot = wgt<AT>(0) * rho0 + d[0];
        rR = cself * tot;
#pragma unroll
        for (int a = 1; a < 9; a++) {
            AT c, vx, vy;
            colour(a, c, vx, vy);
            const AT fa = wgt<AT>(a) * rho0 + d[a];
            rR += c * fa + wgt<AT>(a) * (AT(EX[a]) * vx + AT(EY[a]) * vy);
            tot += fa;
        }
        rB = tot - rR;
    } else {
        AT cs[9], vsx[9], vsy[9];
        cs[0] = cself;
        vsx[0] = vsy[0] = AT(0);
#pragma unroll
        for (int a = 1; a < 9; a++) {
            if (pull_outside(nb, a)) {  // completed below
                cs[a] = cself;
                vsx[a] = vsy[a] = AT(0);
            } else if (m & (1u << (OPP[a] - 1))) {  // half-way bounce-back
                if (!BOUNCED) d[a] = Codec<T>::load(A.fin + OPP[a] * A.plane + self, OPP[a]);
                cs[a] = cself;
                vsx[a] = -vxs;
                vsy[a] = -vys;
            } else {
                colour(a, cs[a], vsx[a], vsy[a]);
            }
        }
        if (nb.lo) {
            // Zou-He velocity inlet on the total f; injected fluid is pure red.
            const AT u = A.inlet[D.io_off + y];
            const AT rho = (rho0 + d[0] + d[2] + d[4] + AT(2) * (d[3] + d[6] + d[7])) / (AT(1) - u);
            const AT ru = rho * u;
            d[1] = d[3] + AT(2.0 / 3.0) * ru;
            d[5] = d[7] - AT(0.5) * (d[2] - d[4]) + AT(1.0 / 6.0) * ru;
            d[8] = d[6] + AT(0.5) * (d[2] - d[4]) + AT(1.0 / 6.0) * ru;
            cs[1] = cs[5] = cs[8] = AT(1);
        }
        if (nb.hi) {
            // Convective outlet f_a <- [f_a(t) + U f_a(x - 1, t + 1)] / (1 + U), coloured with
            // this node's red fraction.
            const AT U = P.outlet_u;
            const uint32_t mm = A.mask[self - 1];
            const AT *h = A.hist_in + (D.io_off + y) * 3;
            const int unk[3] = {3, 6, 7};
#pragma unroll
            for (int q = 0; q < 3; q++) {
                const int a = unk[q];
                AT v = h[q];
                if (!(mm & SELF_SOLID)) {
                    // post-streaming f_a of the neighbour (x - 1, y): from (x, y - e_y) or bounced
                    const AT inner =
                        (mm & (1u << (OPP[a] - 1)))
                            ? Codec<T>::load(A.fin + OPP[a] * A.plane + self - 1, OPP[a])
                            : Codec<T>::load(A.fin + a * A.plane + nb.row[1 - EY[a]] + x, a);
                    v = (v + U * inner) / (AT(1) + U);
                }
                d[a] = v;
            }
        }
        // rho_B as the total minus rho_R: exactly 0 where every source is pure red (c = 1,
        // v = 0), and rho_R exactly 0 where every source is pure blue
        AT tot = AT(0);
#pragma unroll
        for (int a = 0; a < 9; a++) {
            const AT fa = wgt<AT>(a) * rho0 + d[a];
            rR += cs[a] * fa + wgt<AT>(a) * (AT(EX[a]) * vsx[a] + AT(EY[a]) * vsy[a]);
            tot += fa;
        }
        rB = tot - rR;
    }
    if (write_hist && nb.hi) {
        AT *h = A.hist_out + (D.io_off + y) * 3;
        h[0] = d[3];
        h[1] = d[6];
        h[2] = d[7];
    }
}

// Gather with colour state from global memory (read-back and reductions).
template <class T, class AT>
__device__ __forceinline__ void gather_global(const StepArgs<T, AT> &A, DomC &D, int x, int y,
                                              uint32_t m, AT d[9], AT &rR, AT &rB) {
    const Nbr nb = make_nbr(D, x, y);
    const size_t self = nb.row[1] + x;
#pragma unroll
    for (int a = 0; a < 9; a++) {
        const size_t src = A.own ? self : pull_src(nb, a);
        d[a] = Codec<T>::load(A.fin + a * A.plane + src, a);
    }
    finish_gather<false>(A, D, x, y, m, nb, false, d, rR, rB, [&](int a, AT &c, AT &vx, AT &vy) {
        const size_t src = (a == 0 || A.own) ? self : pull_src(nb, a);
        c = A.cin[src];
        vx = A.own ? AT(0) : A.vxin[src];
        vy = A.own ? AT(0) : A.vyin[src];
    });
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

// MRT collision with Guo forcing (Eqs. 1, 2, 8 in moment space) of the deviations d (f = w rho0
// + d), force F, local colour indicator rN; returns the post-collision deviations in o.
template <class AT>
__device__ __forceinline__ void collide(DomC &D, const AT d[9], AT Fx, AT Fy, AT rN,
                                        AT o[9], AT &rho_out, AT &ux_out, AT &uy_out) {
    ParC<AT> &P = par(D, AT());
    const AT rho0 = P.rho0;
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
    const AT inv_rho = rcp(rho);
    const AT ux = (jx + AT(0.5) * Fx) * inv_rho;
    const AT uy = (jy + AT(0.5) * Fy) * inv_rho;
    // Eqs. 18 and 5: 1/nu interpolated in rho^N, tau = 3 nu + 1/2, s_nu = 1/tau
    const AT inv_nu = (AT(1) + rN) * P.inv2nu_r + (AT(1) - rN) * P.inv2nu_b;
    const AT sv = inv_nu * rcp(AT(3) + AT(0.5) * inv_nu);
    const AT se = P.s_e, seps = P.s_eps, sq = P.s_q;

    const AT uu = ux * ux + uy * uy;
    const AT r3uu = AT(3) * rho * uu;
    const AT uF = ux * Fx + uy * Fy;
    const AT p0 = drho;
    const AT p1 = m1 - se * (m1 + AT(2) * drho - r3uu) + P.ke * uF;
    const AT p2 = m2 - seps * (m2 - drho + r3uu) - P.keps * uF;
    const AT p3 = rho * ux + AT(0.5) * Fx;
    const AT p4 = m4 - sq * (m4 + rho * ux) - P.kq * Fx;
    const AT p5 = rho * uy + AT(0.5) * Fy;
    const AT p6 = m6 - sq * (m6 + rho * uy) - P.kq * Fy;
    const AT p7 = m7 - sv * (m7 - rho * (ux * ux - uy * uy)) +
                  (AT(1) - AT(0.5) * sv) * (AT(2) * (ux * Fx - uy * Fy));
    const AT p8 = m8 - sv * (m8 - rho * ux * uy) + (AT(1) - AT(0.5) * sv) * (ux * Fy + uy * Fx);
    // M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
    const AT a0 = p0 * AT(1.0 / 9.0), a1 = p1 * AT(1.0 / 36.0), a2 = p2 * AT(1.0 / 36.0);
    const AT a3 = p3 * AT(1.0 / 6.0), a4 = p4 * AT(1.0 / 12.0);
    const AT a5 = p5 * AT(1.0 / 6.0), a6 = p6 * AT(1.0 / 12.0);
    const AT a7 = p7 * AT(0.25), a8 = p8 * AT(0.25);
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
    rho_out = rho;
    ux_out = ux;
    uy_out = uy;
}

// Work item of block b: blocks are dealt round-robin to the 8 XCDs, so give each XCD a
// contiguous run of items (adjacent strips of a domain share halo columns in its L2).
__device__ __forceinline__ int item_of_block(int b, int n) {
    const int q = n >> 3, rem = n & 7, xcd = b & 7, k = b >> 3;
    return xcd * q + min(xcd, rem) + k;
}

// --------------------------------------------------------------------- step kernel
// ------------------------------------------------------------------ buffer access
// The step kernel streams populations and colour state through buffer resources: a uniform
// descriptor (base, extent below 2^31 bytes), a uniform plane offset and a per-lane byte offset.
// A lane with nothing to move passes NOWHERE, beyond every extent: the hardware then drops the
// store, or returns 0 for the load, without touching memory.  Every wavefront thus issues the
// same vector-memory instructions on every path through a loop iteration, so the compiler can
// wait for exactly the loads a stage consumes; a skipped store would otherwise leave it
// counting as if the prefetch were the newest access and wait for every store in flight.
constexpr uint32_t NOWHERE = 0x80000000u;
using Rsrc = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ Rsrc make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             0x00020000);
}

template <class V>
struct Buf;
template <>
struct Buf<double> {
    __device__ static double load(Rsrc r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    }
    __device__ static void store(Rsrc r, uint32_t vo, uint32_t so, double v) {
        using B = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(B, v), r, vo, so, 0);
    }
};
template <>
struct Buf<float> {
    __device__ static float load(Rsrc r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    __device__ static void store(Rsrc r, uint32_t vo, uint32_t so, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, vo, so, 0);
    }
};
// Two consecutive values (the interleaved wall normal of a node) in one load.
template <class V>
struct Pair {
    V x, y;
};
// (The whole loaded vector is bit-cast: a bit-cast of one element of it, as in
// __builtin_bit_cast(float, v[1]), was compiled as a read of element 0.)
__device__ __forceinline__ Pair<float> load_pair(Rsrc r, uint32_t vo, float) {
    return __builtin_bit_cast(Pair<float>, __builtin_amdgcn_raw_buffer_load_b64(r, vo, 0, 0));
}
__device__ __forceinline__ Pair<double> load_pair(Rsrc r, uint32_t vo, double) {
    return __builtin_bit_cast(Pair<double>, __builtin_amdgcn_raw_buffer_load_b128(r, vo, 0, 0));
}

template <>
struct Buf<__half> {
    __device__ static __half load(Rsrc r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0));
    }
    __device__ static void store(Rsrc r, uint32_t vo, uint32_t so, __half v) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, vo, so, 0);
    }
};
template <>
struct Buf<C16> {
    __device__ static C16 load(Rsrc r, uint32_t vo, uint32_t so) {
        return C16{__builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0)};
    }
    __device__ static void store(Rsrc r, uint32_t vo, uint32_t so, C16 v) {
        __builtin_amdgcn_raw_buffer_store_b16(v.bits, r, vo, so, 0);
    }
};
// Store the lower half of a word (the form the 16-bit encode_sr functions return).
__device__ __forceinline__ void store_lo16(Rsrc r, uint32_t vo, uint32_t so, uint32_t w) {
    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)w, r, vo, so, 0);
}
template <>
struct Buf<uint16_t> {
    __device__ static uint16_t load(Rsrc r, uint32_t vo, uint32_t so) {
        return __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0);
    }
};

// ------------------------------------------------------------------ the step kernel
// R x C wavefronts per block: R tile rows, each C wavefronts (64 C columns) wide.  In iteration
// r the block runs stages B..E on
// rows r + R - 1 + w, r + R - 2 + w, r + R - 3 + w and r + w (w = wavefront), then stage A of
// the next iteration's rows r + 2R + w, and issues the loads for the stage A after that.  Stage E
// of a row runs on the thread that gathered the row one iteration earlier.  LDS rings hold 2R
// rows.  WV: some domain of the launch uses a wetting variant (Sec. III A); without it the
// variant branches are compiled out.
template <class T, int R, int C, bool WV>
__global__ __launch_bounds__(TILE_LANES *R *C, sizeof(typename Codec<T>::AT) == 4 ? 4 : 2) void step_kernel(const StepArgs<T, typename Codec<T>::AT> A) {
    using AT = typename Codec<T>::AT;
    constexpr int Q = 2 * R;
    constexpr int TL = TILE_LANES * C;  // columns of the window: C wavefronts side by side
    constexpr uint32_t SB = sizeof(T), CB = sizeof(AT);
    // Column halo: with FP32 arithmetic every lane gathers, and the colour state of the two
    // columns just outside the window sits in two extra LDS columns (GO = 1), loaded by lanes 0
    // and 1; with FP64 arithmetic the outermost lanes hold it (their extra registers would cost
    // the FP64 kernel an occupancy step).
    constexpr int HX = sizeof(AT) == 8 ? HALO_X64 : HALO_X32;
    constexpr int GO = HX == HALO_X32 ? 1 : 0;
    __shared__ AT s_rn[Q][TL];
    __shared__ AT s_nx[Q][TL], s_ny[Q][TL];
    __shared__ AT s_gx[Q][TL], s_gy[Q][TL];
    __shared__ AT s_c[Q][TL + 2 * GO], s_vx[Q][TL + 2 * GO], s_vy[Q][TL + 2 * GO];
    __shared__ AT s_wx[Q][TL], s_wy[Q][TL];
    __shared__ uint16_t s_m[Q][TL];
    // per row slot and wavefront column: the row has an outermost solid node in that column
    __shared__ int s_wall[Q][C];

    // work item: wave-uniform
    const WorkItem *itp = A.items + item_of_block(blockIdx.x, A.n_items);
    const int dom = __builtin_amdgcn_readfirstlane(itp->dom);
    const int x0 = __builtin_amdgcn_readfirstlane(itp->x0);
    const int y0 = __builtin_amdgcn_readfirstlane(itp->y0), y1 = __builtin_amdgcn_readfirstlane(itp->y1);
    DomC &D = *(DomC *)(A.doms + dom);
    // the wavefront index is uniform within a wavefront: row indices, row-range tests and LDS
    // row slots then live in scalar registers
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / TL);
    const int lane = threadIdx.x % TL;
    const int base = x0 - HX;
    const int X = base + lane;
    // Node column of the lane: periodic in x, or clamped to the edge columns of an open x axis.
    // The x-1 / x+1 stencil neighbours are always the adjacent lanes.  At an open axis the
    // stencil is clamped, so the lanes beyond an edge column stand for that edge node: after
    // each stage that writes a stencil field they copy the edge lane's value (edge_lane >= 0),
    // which only work items touching an open edge do.
    const int xe = D.open_x ? min(max(X, 0), D.nx - 1) : wrap(X, D.nx);
    const bool edge_item = D.open_x && (base < 0 || base + TL > D.nx);
    const int edge_lane = xe != X && D.open_x ? xe - base : -1;
    const int lanes_of[3] = {lane - 1, lane, lane + 1};
    const bool out_lane = lane >= HX && lane < TL - HX && X < D.nx;
    const bool gather_lane = GO || (lane >= 1 && lane < TL - 1);
    // node column of the ghost colour-state column a lane loads (lane 0: left, lane 1: right)
    const int xg = lane == 0 ? base - 1 : base + TL;
    const int xge = D.open_x ? min(max(xg, 0), D.nx - 1) : wrap(xg, D.nx);
    ParC<AT> &P = par(D, AT());
    const AT eps = P.eps;
    const bool rec_cl = A.diag && A.cl_count != nullptr && dom == A.cl_dom;
    const bool scheme_b = WV && (D.wetting & WET_SCHEME_B);
    const bool surface_energy = WV && (D.wetting & WET_SURFACE_ENERGY);
    const int r_first = y0 - HALO + 1 - R;  // first stage A row is y0 - 4

    // a diagnostic launch writes no state (zero extents drop every store) but the velocity
    const Rsrc f_in = make_rsrc(A.fin, A.f_set_bytes), f_out = make_rsrc(A.fout, A.diag ? 0u : A.f_set_bytes);
    // a diagnostic launch writes (u_x, u_y) through the colour-state stores: their resource is
    // then the velocity buffer, whose two-plane extent drops the third store
    const Rsrc c_in = make_rsrc(A.cin, 3 * A.c_plane_bytes);
    const Rsrc c_out = A.diag ? make_rsrc(A.u_out, 2 * A.c_plane_bytes) : make_rsrc(A.cout, 3 * A.c_plane_bytes);
    const Rsrc r_mask = make_rsrc(A.mask, (uint32_t)A.plane * 2u);
    const Rsrc r_ns = make_rsrc(A.ns, A.ns_bytes);
    const uint32_t FP = A.f_plane_bytes, CP = A.c_plane_bytes;

    auto row_ok_a = [&](int y) { return y >= y0 - HALO + 1 && y < y1 + HALO - 1; };
    auto row_ok_c = [&](int y) { return y >= y0 - HALO && y < y1 + HALO; };
    auto node_of = [&](int y) {  // node index of (xe, y), y periodic
        return (uint32_t)D.off + (uint32_t)wrap(y, D.ny) * (uint32_t)D.nx + (uint32_t)xe;
    };

    // Prefetched inputs of one stage A row ya: pulled populations (pulls from solid nodes
    // redirected to the node's own opposite population), its class word and the wall normal on
    // outermost fluid nodes; qm carries the class word of the row, loaded by the previous
    // prefetch.  The set is issued one iteration before its stage A; an iteration issues 26
    // vector memory operations (3 colour loads, 12 stores, 11 prefetch loads).  (A second set
    // issued two iterations ahead measured no faster, and the compiler's waits for it were not
    // exact.)  The colour state that stage D puts into LDS for a stage A row is loaded at the
    // top of the iteration before: vector memory instructions complete in order, stores
    // included, so it then has a full iteration (and never waits for the stores of the stage E
    // in between).  Two colour register sets alternate between iterations (the loop is unrolled
    // twice).
    struct Pre {
        T f[9];
        uint32_t m;
        AT wx, wy;
    };
    Pre pre;
#pragma unroll
    for (int a = 0; a < 9; a++) pre.f[a] = T{};
    pre.m = SELF_SOLID;
    pre.wx = pre.wy = AT(0);
    uint32_t qm = 0;
    struct Colour {
        AT c, vx, vy;
        AT gc, gvx, gvy;  // ghost column (GO only)
    };
    Colour cset[2] = {{AT(0), AT(0), AT(0), AT(0), AT(0), AT(0)}, {AT(0), AT(0), AT(0), AT(0), AT(0), AT(0)}};
    auto load_colour = [&](int yc, Colour &cs) {
        const bool ok = row_ok_c(yc);
        const uint32_t vo = ok ? node_of(yc) * CB : NOWHERE;
        cs.c = Buf<AT>::load(c_in, vo, 0);
        cs.vx = Buf<AT>::load(c_in, vo, CP);
        cs.vy = Buf<AT>::load(c_in, vo, 2 * CP);
        if constexpr (GO) {
            const uint32_t vg = ok && lane < 2
                                    ? ((uint32_t)D.off + (uint32_t)wrap(yc, D.ny) * (uint32_t)D.nx + (uint32_t)xge) * CB
                                    : NOWHERE;
            cs.gc = Buf<AT>::load(c_in, vg, 0);
            cs.gvx = Buf<AT>::load(c_in, vg, CP);
            cs.gvy = Buf<AT>::load(c_in, vg, 2 * CP);
        }
    };
    auto load_mask = [&](int y) {
        qm = Buf<uint16_t>::load(r_mask, row_ok_a(y) ? node_of(y) * 2u : NOWHERE, 0);
    };
    // Column part of the pull offsets (x - 1, x, x + 1; NOWHERE outside the gather lanes), for
    // the prefetch's fast path.
    uint32_t colv[3];
    {
        const Nbr nb0 = make_nbr(D, xe, 0);
#pragma unroll
        for (int k = 0; k < 3; k++) colv[k] = gather_lane ? (uint32_t)nb0.col[k] * SB : NOWHERE;
    }
    auto prefetch = [&](int ya, Pre &p) {
        const bool ok = row_ok_a(ya);
        const uint32_t m = ok ? qm : SELF_SOLID;
        Nbr nb = make_nbr(D, xe, wrap(ya, D.ny));
        // Fast path: no node of the tile row is solid or has a solid neighbour (nothing bounces,
        // every gather lane pulls), the state is not a snapshot and the tile has no open edge.
        // Then a pull's offset is the lane's column plus a wave-uniform row and plane offset,
        // with no vector arithmetic per population.  The branch only chooses offsets: one set
        // of loads follows, so the waits after it stay exact.  Only the FP32-arithmetic kernels
        // take it: they are bound by vector instruction issue; the FP64 kernel is not, and the
        // extra registers would cost it an occupancy step.
        const bool fast = sizeof(AT) == 4 && ok && !A.own && !edge_item &&
                          __builtin_amdgcn_ballot_w64((m & (SELF_SOLID | 0xFFu)) != 0u) == 0;
        uint32_t vo[9], so[9], vw;
        if (fast) {
            vw = NOWHERE;
#pragma unroll
            for (int a = 0; a < 9; a++) {
                vo[a] = colv[1 - EX[a]];
                so[a] = (uint32_t)a * FP + (uint32_t)nb.row[1 - EY[a]] * SB;
            }
        } else {
            const bool act = gather_lane && !(m & SELF_SOLID);
            const uint32_t self = (uint32_t)nb.row[1] + (uint32_t)xe;
            vw = act && (m & FLUID_BND) ? self * (2 * CB) : NOWHERE;
            // snapshot state: every population is the node's own, none bounces
            const uint32_t solid_nbrs = A.own ? 0u : m;
            if (A.own) {
                nb.row[0] = nb.row[2] = nb.row[1];
                nb.col[0] = nb.col[2] = xe;
                nb.lo = nb.hi = false;
            }
#pragma unroll
            for (int a = 0; a < 9; a++) {
                // Direction a and its opposite share the plane offset of the lower of the two;
                // the per-lane offset adds two planes for the higher one (opposites are 2 apart).
                const int lo = a < OPP[a] ? a : OPP[a];
                const uint32_t up = a == lo ? 0u : 2u * FP;
                uint32_t v = (uint32_t)pull_src(nb, a) * SB + up;
                if (a > 0 && !pull_outside(nb, a) && (solid_nbrs & (1u << (OPP[a] - 1))))
                    v = self * SB + (2u * FP - up);
                vo[a] = act ? v : NOWHERE;
                so[a] = (uint32_t)lo * FP;
            }
        }
        const Pair<AT> wn = load_pair(r_ns, vw, AT());
        p.wx = wn.x;
        p.wy = wn.y;
#pragma unroll
        for (int a = 0; a < 9; a++) p.f[a] = Buf<T>::load(f_in, vo[a], so[a]);
        p.m = m;
        load_mask(ya + R);
    };
    // colour row yc into the LDS ring
    auto put_colour = [&](int yc, const Colour &cs) {
        const int sl = yc & (Q - 1);
        s_c[sl][lane + GO] = cs.c;
        s_vx[sl][lane + GO] = cs.vx;
        s_vy[sl][lane + GO] = cs.vy;
        if constexpr (GO) {
            if (lane < 2) {
                const int gl = lane == 0 ? 0 : TL + 1;
                s_c[sl][gl] = cs.gc;
                s_vx[sl][gl] = cs.gvx;
                s_vy[sl][gl] = cs.gvy;
            }
        }
    };
    // one row of outputs: populations, then the colour state (c, vx, vy)
    auto store_row = [&](uint32_t vf, uint32_t vc, const AT (&o)[9], AT c, AT bx, AT by) {
        const uint32_t rb = sizeof(T) == 2 ? round_bits(vf - (uint32_t)D.off * SB, o[0]) : 0u;
#pragma unroll
        for (int a = 0; a < 9; a++) {
            if constexpr (sizeof(T) == 2)
                store_lo16(f_out, vf, (uint32_t)a * FP, Codec<T>::encode_sr(o[a], a, rb));
            else
                Buf<T>::store(f_out, vf, (uint32_t)a * FP, Codec<T>::encode(o[a], a));
        }
        Buf<AT>::store(c_out, vc, 0, c);
        Buf<AT>::store(c_out, vc, CP, bx);
        Buf<AT>::store(c_out, vc, 2 * CP, by);
    };

    auto replicate = [&](AT (*f)[TL], int sl) {
        if (edge_item && edge_lane >= 0) f[sl][lane] = f[sl][edge_lane];
    };

    AT d[9], dn[9];
    AT rR = AT(0), rB = AT(0), rN = AT(0), rRn = AT(0), rBn = AT(0), rNn = AT(0);
#pragma unroll
    for (int a = 0; a < 9; a++) d[a] = dn[a] = AT(0);

    // ---- A: gather, densities, colour indicator of row ya into LDS and dn / rRn / rBn / rNn
    auto stage_a = [&](int ya, const Pre &p) {
        const int sl = ya & (Q - 1);
        const uint32_t m = p.m;
        AT rn = AT(0);
        // decoded on every lane (values of lanes without an output node are never stored):
        // a path that left the prefetched registers unread would make the compiler take them
        // as possibly in flight, and wait for the whole prefetch wherever it reuses one
#pragma unroll
        for (int a = 0; a < 9; a++) dn[a] = Codec<T>::decode(p.f[a], a);
        if (gather_lane && !(m & SELF_SOLID)) {
            const int yw = wrap(ya, D.ny);
            const Nbr nb = make_nbr(D, xe, yw);
            finish_gather<true>(A, D, xe, yw, m, nb, !A.diag, dn, rRn, rBn,
                                [&](int a, AT &c, AT &vx, AT &vy) {
                                    const int s2 = (ya - EY[a]) & (Q - 1);
                                    const int l2 = lanes_of[1 - EX[a]] + GO;
                                    c = s_c[s2][l2];
                                    vx = s_vx[s2][l2];
                                    vy = s_vy[s2][l2];
                                });
            rn = colour_indicator(rRn, rBn);
            rNn = rn;
        }
        s_m[sl][lane] = (uint16_t)m;
        s_rn[sl][lane] = rn;
        s_wx[sl][lane] = p.wx;
        s_wy[sl][lane] = p.wy;
        replicate(s_rn, sl);
        const bool wall = __builtin_amdgcn_ballot_w64((m & SOLID_BND) != 0) != 0;
        if (lane % TILE_LANES == 0) s_wall[sl][lane / TILE_LANES] = wall;
    };
    // Stages B and D change only outermost solid nodes; an iteration whose B (or D) rows have
    // none skips that stage and its barrier.  Every wavefront reads the same flags after a
    // barrier, so the whole block takes the same branch.
    auto any_wall = [&](int ya) {
        int f = 0;
#pragma unroll
        for (int y = 0; y < R; y++)
#pragma unroll
            for (int k = 0; k < C; k++) f |= s_wall[(ya + y) & (Q - 1)][k];
        return __builtin_amdgcn_readfirstlane(f) != 0;
    };

    // prologue: colour rows r_first + R - 1 .. r_first + 2R, stage A of rows r_first + R + w
    load_mask(r_first + R + w);
    if (w < 2) {
        load_colour(r_first + R - 1 + w, cset[0]);
        put_colour(r_first + R - 1 + w, cset[0]);
    }
    load_colour(r_first + R + 1 + w, cset[0]);
    prefetch(r_first + R + w, pre);
    put_colour(r_first + R + 1 + w, cset[0]);
    __syncthreads();
    stage_a(r_first + R + w, pre);
    // the colour rows of the first iteration's stage D and the first prefetch, with as many
    // (dropped) stores in between as the loop issues there, so that the waits in the first
    // iteration are the same as in every later one
    load_colour(r_first + 2 * R + 1 + w, cset[1]);
    store_row(NOWHERE, NOWHERE, d, rR, rB, rN);
    prefetch(r_first + 2 * R + w, pre);

    // One iteration; par selects the colour register sets.
    auto iteration = [&](int r_, auto par_) __attribute__((always_inline)) {
        constexpr int par = decltype(par_)::value;
        // opaque to the compiler's induction analysis: with the loop stepping 2R over rings of
        // 2R rows every ring slot would look loop-invariant and be hoisted into registers
        const int r = __builtin_amdgcn_readfirstlane(r_);
        load_colour(r + 3 * R + 1 + w, cset[par]);  // for the next iteration's stage D
        __syncthreads();
        // scheme (b) has no virtual normals: stage D is skipped on every row
        const bool do_b = any_wall(r + R - 1), do_d = !scheme_b && any_wall(r + R - 3);
        if (do_b) {
            // ---- B: virtual colour indicator on outermost solid nodes (Eq. 29)
            {
                const int yb = r + R - 1 + w;
                const int sl = yb & (Q - 1);
                if (lane >= HX - 3 && lane < TL - (HX - 3) && yb >= y0 - HALO + 2 && yb < y1 + HALO - 2) {
                    const uint32_t m = s_m[sl][lane];
                    if ((m & SOLID_BND) && surface_energy) {
                        s_rn[sl][lane] = P.cos_t;  // surface-energy rule
                    } else if (m & SOLID_BND) {
                        AT num = AT(0), den = AT(0);
    #pragma unroll
                        for (int a = 1; a < 9; a++) {
                            if (m & (1u << (a - 1))) continue;
                            const AT wa = wgt<AT>(a);
                            num += wa * s_rn[(yb + EY[a]) & (Q - 1)][lanes_of[EX[a] + 1]];
                            den += wa;
                        }
                        s_rn[sl][lane] = num * rcp(den);
                    }
                }
                replicate(s_rn, sl);
            }
            __syncthreads();
        }
        // ---- C: colour gradient (Eq. 28), wetting correction, interface normal (Eq. 22)
        {
            const int yc = r + R - 2 + w;
            const int sl = yc & (Q - 1);
            if (lane >= HX - 2 && lane < TL - (HX - 2) && yc >= y0 - HALO + 3 && yc < y1 + HALO - 3) {
                const uint32_t m = s_m[sl][lane];
                AT gx = AT(0), gy = AT(0), nx = AT(0), ny = AT(0);
                if (!(m & SELF_SOLID)) {
                    {
                        AT sx = AT(0), sy = AT(0);
#pragma unroll
                        for (int a = 1; a < 9; a++) {
                            const AT v = s_rn[(yc + EY[a]) & (Q - 1)][lanes_of[EX[a] + 1]];
                            if (EX[a]) sx = acc_nc(sx, wgt<AT>(a), v, EX[a]);
                            if (EY[a]) sy = acc_nc(sy, wgt<AT>(a), v, EY[a]);
                        }
                        gx = AT(3) * sx;
                        gy = AT(3) * sy;
                    }
                    // contact-line list: each node is recorded by the tile that outputs it
                    if (rec_cl && (m & FLUID_BND) && out_lane && yc >= y0 && yc < y1 &&
                        fsqrt(gx * gx + gy * gy) > eps) {
                        const int k = atomicAdd(A.cl_count, 1);
                        if (k < A.cl_cap) A.cl_list[k] = yc * D.nx + X;
                    }
                    if ((m & FLUID_BND) && !surface_energy)
                        wetting_correct(s_wx[sl][lane], s_wy[sl][lane], P.cos_t, P.sin_t, eps, gx, gy);
                    const AT g = fsqrt(gx * gx + gy * gy);
                    if (g > eps) unit_normal(gx, gy, g, nx, ny);
                }
                s_gx[sl][lane] = gx;
                s_gy[sl][lane] = gy;
                s_nx[sl][lane] = nx;
                s_ny[sl][lane] = ny;
            }
            replicate(s_nx, sl);
            replicate(s_ny, sl);
        }
        if (do_d) {
            __syncthreads();
            // ---- D: virtual interface normals on outermost solid nodes (Eq. 29, second BC)
            {
                const int yd = r + R - 3 + w;
                const int sl = yd & (Q - 1);
                if (lane >= HX - 1 && lane < TL - (HX - 1) && yd >= y0 - 1 && yd < y1 + 1) {
                    const uint32_t m = s_m[sl][lane];
                    if (m & SOLID_BND) {
                        AT numx = AT(0), numy = AT(0), den = AT(0);
    #pragma unroll
                        for (int a = 1; a < 9; a++) {
                            if (m & (1u << (a - 1))) continue;
                            const AT wa = wgt<AT>(a);
                            const int s2 = (yd + EY[a]) & (Q - 1);
                            const int l2 = lanes_of[EX[a] + 1];
                            numx += wa * s_nx[s2][l2];
                            numy += wa * s_ny[s2][l2];
                            den += wa;
                        }
                        const AT iden = rcp(den);
                        s_nx[sl][lane] = numx * iden;
                        s_ny[sl][lane] = numy * iden;
                    }
                }
                replicate(s_nx, sl);
                replicate(s_ny, sl);
            }
        }
        // colour row for the coming stage A (loaded at the top of the last iteration)
        put_colour(r + 2 * R + 1 + w, cset[1 - par]);
        __syncthreads();
        // ---- E: curvature (Eq. 13), force (Eq. 10), collision, recolouring state (Eq. 14)
        {
            const int ye = r + w;
            const int sl = ye & (Q - 1);
            // Lanes without an output node store to NOWHERE, so their values are never written;
            // they start from registers that die here, which costs no moves.
            AT o[9], c = rR, bx = rB, by = rN, ux = rR, uy = rB;
#pragma unroll
            for (int a = 0; a < 9; a++) o[a] = d[a];
            uint32_t vf = NOWHERE, vc = NOWHERE;
            const uint32_t me = s_m[sl][lane];
            if (out_lane && ye >= y0 && ye < y1 && !(me & SELF_SOLID)) {
                AT dxnx = AT(0), dynx = AT(0), dxny = AT(0), dyny = AT(0);
                if (scheme_b && (me & FLUID_BND)) {
                    // Eq. 48: weighted mean of the differences to the fluid neighbours
                    const AT nx0 = s_nx[sl][lane], ny0 = s_ny[sl][lane];
                    AT den = AT(0);
#pragma unroll
                    for (int a = 1; a < 9; a++) {
                        if (me & (1u << (a - 1))) continue;
                        const int s2 = (ye + EY[a]) & (Q - 1);
                        const int l2 = lanes_of[EX[a] + 1];
                        const AT vx = s_nx[s2][l2] - nx0, vy = s_ny[s2][l2] - ny0;
                        if (EX[a]) {
                            dxnx += wgt<AT>(a) * vx * AT(EX[a]);
                            dxny += wgt<AT>(a) * vy * AT(EX[a]);
                        }
                        if (EY[a]) {
                            dynx += wgt<AT>(a) * vx * AT(EY[a]);
                            dyny += wgt<AT>(a) * vy * AT(EY[a]);
                        }
                        den += wgt<AT>(a);
                    }
                    const AT iden = rcp(den);
                    dxnx *= iden;
                    dynx *= iden;
                    dxny *= iden;
                    dyny *= iden;
                } else {
#pragma unroll
                    for (int a = 1; a < 9; a++) {
                        const int s2 = (ye + EY[a]) & (Q - 1);
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
                const AT Fx = P.half_sigma * kappa * gx;
                const AT Fy = P.half_sigma * kappa * gy;
                AT rho;
                collide(D, d, Fx, Fy, rN, o, rho, ux, uy);
                const AT rs = rR + rB;
                c = quotient(rR, rs);
                const AT b = P.beta * rB * c;
                bx = b * nx;
                by = b * ny;
                const uint32_t nd = node_of(ye);
                vf = nd * SB;
                vc = nd * CB;
                if (!isfinite(rho + ux + uy)) atomicOr(A.flag, 1);  // any NaN or overflow
            }
            if (A.diag) {
                c = ux;
                bx = uy;
            }
            store_row(vf, vc, o, c, bx, by);
        }
#pragma unroll
        for (int a = 0; a < 9; a++) d[a] = dn[a];
        rR = rRn;
        rB = rBn;
        rN = rNn;
        // Stage A of the next iteration, without a barrier: it writes s_m / s_rn rows
        // r + 2R .. r + 3R - 1, which alias rows r .. r + R - 1; of those, stage E reads only
        // s_m of its own row, written by its own wavefront.  The colour rows it reads were
        // put into LDS after stage D, before the last barrier.
        stage_a(r + 2 * R + w, pre);
        prefetch(r + 3 * R + w, pre);
    };
    // Both exits test the row bound themselves: an exit merged into a shared loop test would
    // put a path from the first half back to the loop head, where the compiler would then take
    // the first half's prefetch as possibly still in flight.  (r_first < y0 < y1.)
    for (int r = r_first;; r += 2 * R) {
        iteration(r, std::integral_constant<int, 0>());
        if (r + R >= y1) break;
        iteration(r + R, std::integral_constant<int, 1>());
        if (r + 2 * R >= y1) break;
    }
}

// --------------------------------------------------- the step kernel with two columns per lane
// Same method, same stages and the same per-node arithmetic as step_kernel, for the storages
// with FP32 arithmetic, but each lane owns two adjacent node columns (an even one and the next)
// of a window 128 columns wide: one wavefront per tile row, 116 output columns and a halo of 6
// on each side (even, so that a lane's two columns are both output or both halo).  Two nodes per
// lane halve the share of halo lanes and of per-lane row overhead (addresses, loop control, ring
// slots), and every population, colour-state and class-word access moves both nodes at once:
// one 4-byte access per 16-bit population pair (8 bytes for FP32), so each vector memory
// instruction carries twice the bytes.  Requires an even nx in every domain (the host falls back
// to step_kernel otherwise), so that a lane's pair never straddles a row end or a periodic seam.
//
// Pulls read the pair (x - e_x, x + 1 - e_x) of row y - e_y in one access; for e_x != 0 that is a
// 2-byte aligned 4-byte access (unaligned global access mode).  Where the two nodes of a lane need
// non-adjacent sources - one of them bounces back from a solid node and the other does not, or the
// pull crosses a periodic seam - the pair access serves the even node and the odd node's value is
// loaded on its own in stage A (rare: curved walls and seam columns; straight walls bounce both).
template <class T>
struct PairIO;
template <>
struct PairIO<C16> {
    using V = uint32_t;
    __device__ static V load(Rsrc r, uint32_t vo, uint32_t so) {
        return __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0);
    }
    __device__ static void store(Rsrc r, uint32_t vo, uint32_t so, V v) {
        __builtin_amdgcn_raw_buffer_store_b32(v, r, vo, so, 0);
    }
    // Sign and 15 exponent-and-fraction bits of each half moved to bits 31 and 12..26 of an FP32
    // word (the same word Codec<C16>::decode forms), by one arithmetic shift and one mask each.
    __device__ static void decode(V v, int a, float &lo, float &hi) {
        const uint32_t l = (uint32_t)((int32_t)(v << 16) >> 4) & 0x87FFF000u;
        const uint32_t h = (uint32_t)((int32_t)v >> 4) & 0x87FFF000u;
        lo = __uint_as_float(l) * Codec<C16>::dec(a);
        hi = __uint_as_float(h) * Codec<C16>::dec(a);
    }
    // stochastic rounding as in step_kernel, with each node's own random bits
    __device__ static V encode(float lo, float hi, int a, uint32_t rlo, uint32_t rhi) {
        return (Codec<C16>::encode_sr(lo, a, rlo) & 0xFFFFu) | (Codec<C16>::encode_sr(hi, a, rhi) << 16);
    }
    __device__ static V zero() { return 0u; }
};
template <>
struct PairIO<__half> {
    using V = uint32_t;
    __device__ static V load(Rsrc r, uint32_t vo, uint32_t so) {
        return __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0);
    }
    __device__ static void store(Rsrc r, uint32_t vo, uint32_t so, V v) {
        __builtin_amdgcn_raw_buffer_store_b32(v, r, vo, so, 0);
    }
    __device__ static void decode(V v, int a, float &lo, float &hi) {
        lo = Codec<__half>::decode(__ushort_as_half((unsigned short)(v & 0xFFFFu)), a);
        hi = Codec<__half>::decode(__ushort_as_half((unsigned short)(v >> 16)), a);
    }
    // stochastic rounding as in step_kernel, with each node's own random bits
    __device__ static V encode(float lo, float hi, int a, uint32_t rlo, uint32_t rhi) {
        return (Codec<__half>::encode_sr(lo, a, rlo) & 0xFFFFu) | (Codec<__half>::encode_sr(hi, a, rhi) << 16);
    }
    __device__ static V zero() { return 0u; }
};
template <>
struct PairIO<float> {
    using V = Pair<float>;
    __device__ static V load(Rsrc r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    }
    __device__ static void store(Rsrc r, uint32_t vo, uint32_t so, V v) {
        using B = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(B, v), r, vo, so, 0);
    }
    __device__ static void decode(V v, int, float &lo, float &hi) {
        lo = v.x;
        hi = v.y;
    }
    __device__ static V encode(float lo, float hi, int, uint32_t, uint32_t) { return V{lo, hi}; }
    __device__ static V zero() { return V{0.0f, 0.0f}; }
};

__device__ __forceinline__ Pair<float> load_f2(Rsrc r, uint32_t vo, uint32_t so) {
    return __builtin_bit_cast(Pair<float>, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
}
__device__ __forceinline__ void store_f2(Rsrc r, uint32_t vo, uint32_t so, float lo, float hi) {
    using B = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(B, Pair<float>{lo, hi}), r, vo, so, 0);
}
struct Quad {
    float a, b, c, d;
};
__device__ __forceinline__ Quad load_f4(Rsrc r, uint32_t vo) {
    return __builtin_bit_cast(Quad, __builtin_amdgcn_raw_buffer_load_b128(r, vo, 0, 0));
}

// Element (plane * plane_elems + node) that node (x, y) with neighbourhood nb and class word m
// needs for direction a: the pull source x - e_a in plane a, the node's own value in plane
// opp(a) for a link from a solid node (half-way bounce-back), the node itself in snapshot mode;
// -1 for a pull across the inlet or the outlet (completed by the boundary condition).
__device__ __forceinline__ long long pull_elem(const Nbr &nb, int x, uint32_t m, int a, bool own,
                                               size_t plane_elems) {
    const size_t self = nb.row[1] + x;
    if (own || a == 0) return (long long)(a * plane_elems + self);
    if (pull_outside(nb, a)) return -1;
    if (m & (1u << (OPP[a] - 1))) return (long long)(OPP[a] * plane_elems + self);
    return (long long)(a * plane_elems + pull_src(nb, a));
}

constexpr int PAIR_HALO = 6;                          // halo columns per side (even)
constexpr int PAIR_COLS = 2 * TILE_LANES;             // window columns
constexpr int PAIR_OUT = PAIR_COLS - 2 * PAIR_HALO;   // output columns of a window
static_assert(PAIR_OUT == 2 * TILE_LANES - 12, "the host's tile_out(cols, 2) strides strips by the pair window's outputs");

template <class T, int R, bool WV>
__global__ __launch_bounds__(TILE_LANES *R, 2) void pair_kernel(const StepArgs<T, float> A) {
    using AT = float;
    using IO = PairIO<T>;
    using PV = typename IO::V;
    constexpr int Q = 2 * R;
    constexpr int TW = PAIR_COLS;
    constexpr uint32_t SB = sizeof(T), CB = sizeof(AT);
    __shared__ AT s_rn[Q][TW];
    __shared__ AT s_nx[Q][TW], s_ny[Q][TW];
    __shared__ AT s_gx[Q][TW], s_gy[Q][TW];
    __shared__ AT s_c[Q][TW], s_vx[Q][TW], s_vy[Q][TW];
    __shared__ AT s_wx[Q][TW], s_wy[Q][TW];
    __shared__ uint16_t s_m[Q][TW];
    __shared__ int s_wall[Q];

    const WorkItem *itp = A.items + item_of_block(blockIdx.x, A.n_items);
    const int dom = __builtin_amdgcn_readfirstlane(itp->dom);
    const int x0 = __builtin_amdgcn_readfirstlane(itp->x0);
    const int y0 = __builtin_amdgcn_readfirstlane(itp->y0), y1 = __builtin_amdgcn_readfirstlane(itp->y1);
    DomC &D = *(DomC *)(A.doms + dom);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / TILE_LANES);
    const int lane = threadIdx.x % TILE_LANES;
    const int base = x0 - PAIR_HALO;
    // the lane's two window columns and node columns (periodic, or clamped at an open x axis)
    int col[2], X[2], xe[2], edge_col[2];
    bool out[2], gath[2];
#pragma unroll
    for (int k = 0; k < 2; k++) {
        col[k] = 2 * lane + k;
        X[k] = base + col[k];
        xe[k] = D.open_x ? min(max(X[k], 0), D.nx - 1) : wrap(X[k], D.nx);
        edge_col[k] = xe[k] != X[k] && D.open_x ? xe[k] - base : -1;
        out[k] = col[k] >= PAIR_HALO && col[k] < TW - PAIR_HALO && X[k] < D.nx;
        // columns beyond an open end take the edge column's stencil values (replicate below),
        // so they gather nothing themselves
        gath[k] = col[k] >= 1 && col[k] < TW - 1 && edge_col[k] < 0;
    }
    // the window reaches past a domain edge (an open end or a periodic seam)
    const bool edge_item = base < 0 || base + TW > D.nx;
    const bool open_edge = D.open_x && edge_item;
    ParC<AT> &P = par(D, AT());
    const AT eps = P.eps;
    const bool rec_cl = A.diag && A.cl_count != nullptr && dom == A.cl_dom;
    const bool scheme_b = WV && (D.wetting & WET_SCHEME_B);
    const bool surface_energy = WV && (D.wetting & WET_SURFACE_ENERGY);
    const int r_first = y0 - HALO + 1 - R;

    const Rsrc f_in = make_rsrc(A.fin, A.f_set_bytes), f_out = make_rsrc(A.fout, A.diag ? 0u : A.f_set_bytes);
    const Rsrc c_in = make_rsrc(A.cin, 3 * A.c_plane_bytes);
    const Rsrc c_out = A.diag ? make_rsrc(A.u_out, 2 * A.c_plane_bytes) : make_rsrc(A.cout, 3 * A.c_plane_bytes);
    const Rsrc r_mask = make_rsrc(A.mask, (uint32_t)A.plane * 2u);
    const Rsrc r_ns = make_rsrc(A.ns, A.ns_bytes);
    const uint32_t FP = A.f_plane_bytes, CP = A.c_plane_bytes;

    auto row_ok_a = [&](int y) { return y >= y0 - HALO + 1 && y < y1 + HALO - 1; };
    auto row_ok_c = [&](int y) { return y >= y0 - HALO && y < y1 + HALO; };
    // node index of the lane's even column in row y (y periodic); the odd column is the next one
    auto node_of = [&](int y) {
        return (uint32_t)D.off + (uint32_t)wrap(y, D.ny) * (uint32_t)D.nx + (uint32_t)xe[0];
    };
    // a clamped lane beyond an open end stands for the edge node in both columns
    const bool clamp_pair = xe[1] != xe[0] + 1;

    struct Pre {
        PV f[9];
        uint32_t m0, m1;   // class words of the two nodes
        uint32_t fix;      // directions whose odd-column value is loaded on its own in stage A
        AT wx0, wy0, wx1, wy1;
    };
    Pre pre;
#pragma unroll
    for (int a = 0; a < 9; a++) pre.f[a] = IO::zero();
    pre.m0 = pre.m1 = SELF_SOLID;
    pre.fix = 0;
    pre.wx0 = pre.wy0 = pre.wx1 = pre.wy1 = AT(0);
    uint32_t qm0 = 0, qm1 = 0;
    struct Colour {
        AT c0, c1, vx0, vx1, vy0, vy1;
    };
    Colour cset[2] = {{}, {}};
    auto load_colour = [&](int yc, Colour &cs) {
        const uint32_t vo = row_ok_c(yc) ? node_of(yc) * CB : NOWHERE;
        const Pair<AT> c = load_f2(c_in, vo, 0), vx = load_f2(c_in, vo, CP), vy = load_f2(c_in, vo, 2 * CP);
        cs.c0 = c.x;
        cs.vx0 = vx.x;
        cs.vy0 = vy.x;
        cs.c1 = clamp_pair ? c.x : c.y;
        cs.vx1 = clamp_pair ? vx.x : vx.y;
        cs.vy1 = clamp_pair ? vy.x : vy.y;
    };
    auto load_mask = [&](int y) {
        const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(r_mask, row_ok_a(y) ? node_of(y) * 2u : NOWHERE, 0, 0);
        qm0 = v & 0xFFFFu;
        qm1 = clamp_pair ? qm0 : v >> 16;
    };
    // fast-path column offsets of the pair pulled along e_x = +1, 0, -1
    uint32_t colv[3];
#pragma unroll
    for (int k = 0; k < 3; k++) colv[k] = (gath[0] || gath[1]) ? (uint32_t)(xe[0] - 1 + k) * SB : NOWHERE;

    auto prefetch = [&](int ya, Pre &p) {
        const bool ok = row_ok_a(ya);
        const uint32_t m0 = ok ? qm0 : SELF_SOLID, m1 = ok ? qm1 : SELF_SOLID;
        const int yw = wrap(ya, D.ny);
        const bool fast = ok && !A.own && !edge_item &&
                          __builtin_amdgcn_ballot_w64(((m0 | m1) & (SELF_SOLID | 0xFFu)) != 0u) == 0;
        uint32_t vo[9], so[9], vw, fix = 0;
        if (fast) {
            vw = NOWHERE;
            const uint32_t row[3] = {
                (uint32_t)D.off + (uint32_t)(yw == 0 ? D.ny - 1 : yw - 1) * (uint32_t)D.nx,
                (uint32_t)D.off + (uint32_t)yw * (uint32_t)D.nx,
                (uint32_t)D.off + (uint32_t)(yw == D.ny - 1 ? 0 : yw + 1) * (uint32_t)D.nx};
#pragma unroll
            for (int a = 0; a < 9; a++) {
                vo[a] = colv[1 - EX[a]];
                so[a] = (uint32_t)a * FP + row[1 - EY[a]] * SB;
            }
        } else {
            const Nbr nb0 = make_nbr(D, xe[0], yw), nb1 = make_nbr(D, xe[1], yw);
            const bool act0 = gath[0] && !(m0 & SELF_SOLID), act1 = gath[1] && !(m1 & SELF_SOLID);
            const uint32_t self0 = (uint32_t)nb0.row[1] + (uint32_t)xe[0];
            vw = (act0 && (m0 & FLUID_BND)) || (act1 && (m1 & FLUID_BND)) ? self0 * (2 * CB) : NOWHERE;
#pragma unroll
            for (int a = 0; a < 9; a++) {
                const long long s0 = act0 ? pull_elem(nb0, xe[0], m0, a, A.own, A.plane) : -1;
                const long long s1 = act1 ? pull_elem(nb1, xe[1], m1, a, A.own, A.plane) : -1;
                long long e;
                if (s0 < 0) {
                    e = s1 < 0 ? -1 : s1 - 1;
                } else {
                    e = s0;
                    if (s1 >= 0 && s1 != s0 + 1) fix |= 1u << a;
                }
                vo[a] = e < 0 ? NOWHERE : (uint32_t)e * SB;
                so[a] = 0;
            }
        }
        const Quad wn = load_f4(r_ns, vw);
        p.wx0 = wn.a;
        p.wy0 = wn.b;
        p.wx1 = wn.c;
        p.wy1 = wn.d;
#pragma unroll
        for (int a = 0; a < 9; a++) p.f[a] = IO::load(f_in, vo[a], so[a]);
        p.m0 = m0;
        p.m1 = m1;
        p.fix = fix;
        load_mask(ya + R);
    };
    auto put_colour = [&](int yc, const Colour &cs) {
        const int sl = yc & (Q - 1);
        s_c[sl][col[0]] = cs.c0;
        s_c[sl][col[1]] = cs.c1;
        s_vx[sl][col[0]] = cs.vx0;
        s_vx[sl][col[1]] = cs.vx1;
        s_vy[sl][col[0]] = cs.vy0;
        s_vy[sl][col[1]] = cs.vy1;
    };
    auto replicate = [&](AT (*f)[TW], int sl) __attribute__((always_inline)) {
        if (open_edge) {
#pragma unroll
            for (int k = 0; k < 2; k++)
                if (edge_col[k] >= 0) f[sl][col[k]] = f[sl][edge_col[k]];
        }
    };

    // populations of the two nodes (indices constant after unrolling, so they stay in registers)
    AT d[2][9], dn[2][9];
    AT rR[2] = {AT(0), AT(0)}, rB[2] = {AT(0), AT(0)}, rN[2] = {AT(0), AT(0)};
    AT rRn[2] = {AT(0), AT(0)}, rBn[2] = {AT(0), AT(0)}, rNn[2] = {AT(0), AT(0)};
#pragma unroll
    for (int a = 0; a < 9; a++) d[0][a] = d[1][a] = dn[0][a] = dn[1][a] = AT(0);

    // ---- A: gather, densities, colour indicator of row ya into LDS and dn / rRn / rBn / rNn
    auto stage_a = [&](int ya, const Pre &p) __attribute__((always_inline)) {
        const int sl = ya & (Q - 1);
#pragma unroll
        for (int a = 0; a < 9; a++) IO::decode(p.f[a], a, dn[0][a], dn[1][a]);
        const int yw = wrap(ya, D.ny);
        if (__builtin_amdgcn_ballot_w64(p.fix != 0u) != 0) {
            // odd-column values whose source is not next to the even column's source
            if (p.fix) {
                const Nbr nb1 = make_nbr(D, xe[1], yw);
#pragma unroll
                for (int a = 0; a < 9; a++)
                    if (p.fix & (1u << a)) {
                        const long long e = pull_elem(nb1, xe[1], p.m1, a, A.own, A.plane);
                        dn[1][a] = Codec<T>::load(A.fin + e, a);
                    }
            }
        }
        const uint32_t ms[2] = {p.m0, p.m1};
        AT rn[2] = {AT(0), AT(0)};
#pragma unroll
        for (int k = 0; k < 2; k++) {
            if (gath[k] && !(ms[k] & SELF_SOLID)) {
                const Nbr nb = make_nbr(D, xe[k], yw);
                const int ck = col[k];
                finish_gather<true>(A, D, xe[k], yw, ms[k], nb, !A.diag, dn[k], rRn[k], rBn[k],
                                    [&](int a, AT &c, AT &vx, AT &vy) {
                                        const int s2 = (ya - EY[a]) & (Q - 1);
                                        const int l2 = ck - EX[a];
                                        c = s_c[s2][l2];
                                        vx = s_vx[s2][l2];
                                        vy = s_vy[s2][l2];
                                    });
                rn[k] = colour_indicator(rRn[k], rBn[k]);
                rNn[k] = rn[k];
            }
        }
        s_m[sl][col[0]] = (uint16_t)p.m0;
        s_m[sl][col[1]] = (uint16_t)p.m1;
        s_rn[sl][col[0]] = rn[0];
        s_rn[sl][col[1]] = rn[1];
        s_wx[sl][col[0]] = p.wx0;
        s_wy[sl][col[0]] = p.wy0;
        s_wx[sl][col[1]] = p.wx1;
        s_wy[sl][col[1]] = p.wy1;
        replicate(s_rn, sl);
        const bool wall = __builtin_amdgcn_ballot_w64(((p.m0 | p.m1) & SOLID_BND) != 0) != 0;
        if (lane == 0) s_wall[sl] = wall;
    };
    auto any_wall = [&](int ya) __attribute__((always_inline)) {
        int f = 0;
#pragma unroll
        for (int y = 0; y < R; y++) f |= s_wall[(ya + y) & (Q - 1)];
        return __builtin_amdgcn_readfirstlane(f) != 0;
    };

    load_mask(r_first + R + w);
    if (w < 2) {
        load_colour(r_first + R - 1 + w, cset[0]);
        put_colour(r_first + R - 1 + w, cset[0]);
    }
    load_colour(r_first + R + 1 + w, cset[0]);
    prefetch(r_first + R + w, pre);
    put_colour(r_first + R + 1 + w, cset[0]);
    __syncthreads();
    stage_a(r_first + R + w, pre);
    load_colour(r_first + 2 * R + 1 + w, cset[1]);
    {
        // as many (dropped) stores as the loop issues between its colour loads and the prefetch
#pragma unroll
        for (int a = 0; a < 9; a++) IO::store(f_out, NOWHERE, (uint32_t)a * FP, IO::zero());
        store_f2(c_out, NOWHERE, 0, AT(0), AT(0));
        store_f2(c_out, NOWHERE, CP, AT(0), AT(0));
        store_f2(c_out, NOWHERE, 2 * CP, AT(0), AT(0));
    }
    prefetch(r_first + 2 * R + w, pre);

    auto iteration = [&](int r_, auto par_) __attribute__((always_inline)) {
        constexpr int par = decltype(par_)::value;
        const int r = __builtin_amdgcn_readfirstlane(r_);
        load_colour(r + 3 * R + 1 + w, cset[par]);
        __syncthreads();
        const bool do_b = any_wall(r + R - 1), do_d = !scheme_b && any_wall(r + R - 3);
        if (do_b) {
            // ---- B: virtual colour indicator on outermost solid nodes (Eq. 29)
            const int yb = r + R - 1 + w;
            const int sl = yb & (Q - 1);
            if (yb >= y0 - HALO + 2 && yb < y1 + HALO - 2) {
#pragma unroll
                for (int k = 0; k < 2; k++) {
                    const int ck = col[k];
                    if (ck >= 2 && ck < TW - 2) {
                        const uint32_t m = s_m[sl][ck];
                        if ((m & SOLID_BND) && surface_energy) {
                            s_rn[sl][ck] = P.cos_t;
                        } else if (m & SOLID_BND) {
                            AT num = AT(0), den = AT(0);
#pragma unroll
                            for (int a = 1; a < 9; a++) {
                                if (m & (1u << (a - 1))) continue;
                                const AT wa = wgt<AT>(a);
                                num += wa * s_rn[(yb + EY[a]) & (Q - 1)][ck + EX[a]];
                                den += wa;
                            }
                            s_rn[sl][ck] = num * rcp(den);
                        }
                    }
                }
            }
            replicate(s_rn, sl);
            __syncthreads();
        }
        // ---- C: colour gradient (Eq. 28), wetting correction, interface normal (Eq. 22)
        {
            const int yc = r + R - 2 + w;
            const int sl = yc & (Q - 1);
            if (yc >= y0 - HALO + 3 && yc < y1 + HALO - 3) {
#pragma unroll
                for (int k = 0; k < 2; k++) {
                    const int ck = col[k];
                    if (ck >= 3 && ck < TW - 3) {
                        const uint32_t m = s_m[sl][ck];
                        AT gx = AT(0), gy = AT(0), nx = AT(0), ny = AT(0);
                        if (!(m & SELF_SOLID)) {
                            AT sx = AT(0), sy = AT(0);
#pragma unroll
                            for (int a = 1; a < 9; a++) {
                                const AT v = s_rn[(yc + EY[a]) & (Q - 1)][ck + EX[a]];
                                if (EX[a]) sx = acc_nc(sx, wgt<AT>(a), v, EX[a]);
                                if (EY[a]) sy = acc_nc(sy, wgt<AT>(a), v, EY[a]);
                            }
                            gx = AT(3) * sx;
                            gy = AT(3) * sy;
                            if (rec_cl && (m & FLUID_BND) && out[k] && yc >= y0 && yc < y1 &&
                                fsqrt(gx * gx + gy * gy) > eps) {
                                const int q = atomicAdd(A.cl_count, 1);
                                if (q < A.cl_cap) A.cl_list[q] = yc * D.nx + X[k];
                            }
                            if ((m & FLUID_BND) && !surface_energy)
                                wetting_correct(s_wx[sl][ck], s_wy[sl][ck], P.cos_t, P.sin_t, eps, gx, gy);
                            const AT g = fsqrt(gx * gx + gy * gy);
                            if (g > eps) unit_normal(gx, gy, g, nx, ny);
                        }
                        s_gx[sl][ck] = gx;
                        s_gy[sl][ck] = gy;
                        s_nx[sl][ck] = nx;
                        s_ny[sl][ck] = ny;
                    }
                }
            }
            replicate(s_nx, sl);
            replicate(s_ny, sl);
        }
        if (do_d) {
            __syncthreads();
            // ---- D: virtual interface normals on outermost solid nodes (Eq. 29, second BC)
            const int yd = r + R - 3 + w;
            const int sl = yd & (Q - 1);
            if (yd >= y0 - 1 && yd < y1 + 1) {
#pragma unroll
                for (int k = 0; k < 2; k++) {
                    const int ck = col[k];
                    if (ck >= 4 && ck < TW - 4) {
                        const uint32_t m = s_m[sl][ck];
                        if (m & SOLID_BND) {
                            AT numx = AT(0), numy = AT(0), den = AT(0);
#pragma unroll
                            for (int a = 1; a < 9; a++) {
                                if (m & (1u << (a - 1))) continue;
                                const AT wa = wgt<AT>(a);
                                const int s2 = (yd + EY[a]) & (Q - 1);
                                numx += wa * s_nx[s2][ck + EX[a]];
                                numy += wa * s_ny[s2][ck + EX[a]];
                                den += wa;
                            }
                            const AT iden = rcp(den);
                            s_nx[sl][ck] = numx * iden;
                            s_ny[sl][ck] = numy * iden;
                        }
                    }
                }
            }
            replicate(s_nx, sl);
            replicate(s_ny, sl);
        }
        put_colour(r + 2 * R + 1 + w, cset[1 - par]);
        __syncthreads();
        // ---- E: curvature (Eq. 13), force (Eq. 10), collision, recolouring state (Eq. 14)
        {
            const int ye = r + w;
            const int sl = ye & (Q - 1);
            const bool row_out = ye >= y0 && ye < y1;
            AT o[2][9];
            AT cst[2], bxs[2], bys[2];
#pragma unroll
            for (int k = 0; k < 2; k++) {
                const int ck = col[k];
                // solid nodes store zero deviations and colour state (their initial values)
                AT c = AT(0), bx = AT(0), by = AT(0), ux = AT(0), uy = AT(0);
#pragma unroll
                for (int a = 0; a < 9; a++) o[k][a] = AT(0);
                const uint32_t me = s_m[sl][ck];
                if (out[k] && row_out && !(me & SELF_SOLID)) {
                    AT dxnx = AT(0), dynx = AT(0), dxny = AT(0), dyny = AT(0);
                    if (scheme_b && (me & FLUID_BND)) {
                        const AT nx0 = s_nx[sl][ck], ny0 = s_ny[sl][ck];
                        AT den = AT(0);
#pragma unroll
                        for (int a = 1; a < 9; a++) {
                            if (me & (1u << (a - 1))) continue;
                            const int s2 = (ye + EY[a]) & (Q - 1);
                            const AT vx = s_nx[s2][ck + EX[a]] - nx0, vy = s_ny[s2][ck + EX[a]] - ny0;
                            if (EX[a]) {
                                dxnx += wgt<AT>(a) * vx * AT(EX[a]);
                                dxny += wgt<AT>(a) * vy * AT(EX[a]);
                            }
                            if (EY[a]) {
                                dynx += wgt<AT>(a) * vx * AT(EY[a]);
                                dyny += wgt<AT>(a) * vy * AT(EY[a]);
                            }
                            den += wgt<AT>(a);
                        }
                        const AT iden = rcp(den);
                        dxnx *= iden;
                        dynx *= iden;
                        dxny *= iden;
                        dyny *= iden;
                    } else {
#pragma unroll
                        for (int a = 1; a < 9; a++) {
                            const int s2 = (ye + EY[a]) & (Q - 1);
                            const AT vx = s_nx[s2][ck + EX[a]], vy = s_ny[s2][ck + EX[a]];
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
                    const AT nx = s_nx[sl][ck], ny = s_ny[sl][ck];
                    const AT gx = s_gx[sl][ck], gy = s_gy[sl][ck];
                    const AT kappa = -nx * nx * dyny - ny * ny * dxnx + nx * ny * (dynx + dxny);
                    const AT Fx = P.half_sigma * kappa * gx;
                    const AT Fy = P.half_sigma * kappa * gy;
                    AT rho;
                    collide(D, d[k], Fx, Fy, rN[k], o[k], rho, ux, uy);
                    const AT rs = rR[k] + rB[k];
                    c = quotient(rR[k], rs);
                    const AT b = P.beta * rB[k] * c;
                    bx = b * nx;
                    by = b * ny;
                    if (!isfinite(rho + ux + uy)) atomicOr(A.flag, 1);
                }
                if (A.diag) {
                    c = ux;
                    bx = uy;
                }
                cst[k] = c;
                bxs[k] = bx;
                bys[k] = by;
            }
            const uint32_t nd = node_of(ye);
            const bool st = out[0] && row_out;
            const uint32_t vf = st ? nd * SB : NOWHERE, vc = st ? nd * CB : NOWHERE;
            const uint32_t vl = vf - (uint32_t)D.off * SB;  // offset within the domain
            const uint32_t rb0 = sizeof(T) == 2 ? round_bits(vl, o[0][0]) : 0u;
            const uint32_t rb1 = sizeof(T) == 2 ? round_bits(vl + SB, o[1][0]) : 0u;
#pragma unroll
            for (int a = 0; a < 9; a++)
                IO::store(f_out, vf, (uint32_t)a * FP, IO::encode(o[0][a], o[1][a], a, rb0, rb1));
            store_f2(c_out, vc, 0, cst[0], cst[1]);
            store_f2(c_out, vc, CP, bxs[0], bxs[1]);
            store_f2(c_out, vc, 2 * CP, bys[0], bys[1]);
        }
#pragma unroll
        for (int a = 0; a < 9; a++) {
            d[0][a] = dn[0][a];
            d[1][a] = dn[1][a];
        }
#pragma unroll
        for (int k = 0; k < 2; k++) {
            rR[k] = rRn[k];
            rB[k] = rBn[k];
            rN[k] = rNn[k];
        }
        stage_a(r + 2 * R + w, pre);
        prefetch(r + 3 * R + w, pre);
    };
    for (int r = r_first;; r += 2 * R) {
        iteration(r, std::integral_constant<int, 0>());
        if (r + R >= y1) break;
        iteration(r + R, std::integral_constant<int, 1>());
        if (r + 2 * R >= y1) break;
    }
}

// ------------------------------------------------------------- decode to FP64 fields
template <class T>
__global__ void read_kernel(const StepArgs<T, typename Codec<T>::AT> A, int dom, uint32_t which,
                            double *out) {
    using AT = typename Codec<T>::AT;
    DomC &D = *(DomC *)(A.doms + dom);
    const size_t nn = (size_t)D.nx * D.ny;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nn;
         i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % D.nx), y = (int)(i / D.nx);
        const uint32_t m = A.mask[D.off + i];
        double fR[9], fB[9], sR = 0.0, sB = 0.0;
#pragma unroll
        for (int a = 0; a < 9; a++) fR[a] = fB[a] = 0.0;
        if (!(m & SELF_SOLID)) {
            // the step's completion of the populations, then the colour source of each one
            const Nbr nb = make_nbr(D, x, y);
            const size_t self = nb.row[1] + x;
            AT d[9], rR, rB;
#pragma unroll
            for (int a = 0; a < 9; a++)
                d[a] = Codec<T>::load(A.fin + a * A.plane + (A.own ? self : pull_src(nb, a)),
                                      a);
            finish_gather<false>(A, D, x, y, m, nb, false, d, rR, rB, [&](int a, AT &c, AT &vx, AT &vy) {
                const size_t src = (a == 0 || A.own) ? self : pull_src(nb, a);
                c = A.cin[src];
                vx = A.own ? AT(0) : A.vxin[src];
                vy = A.own ? AT(0) : A.vyin[src];
            });
            const AT cself = A.cin[self];
            const AT vxs = A.own ? AT(0) : A.vxin[self], vys = A.own ? AT(0) : A.vyin[self];
#pragma unroll
            for (int a = 0; a < 9; a++) {
                AT cs, vsx, vsy;
                if (A.own || a == 0) {
                    cs = cself;
                    vsx = vsy = AT(0);
                } else if (pull_outside(nb, a)) {
                    cs = nb.lo ? AT(1) : cself;  // inlet injects red; outlet keeps the node's
                    vsx = vsy = AT(0);
                } else if (m & (1u << (OPP[a] - 1))) {
                    cs = cself;
                    vsx = -vxs;
                    vsy = -vys;
                } else {
                    const size_t src = pull_src(nb, a);
                    cs = A.cin[src];
                    vsx = A.vxin[src];
                    vsy = A.vyin[src];
                }
                const double fa = wgt<double>(a) * D.d.rho0 + (double)d[a];
                const double t = wgt<double>(a) * (EX[a] * (double)vsx + EY[a] * (double)vsy);
                fR[a] = (double)cs * fa + t;
                fB[a] = (1.0 - (double)cs) * fa - t;
                sR += fR[a];
                sB += fB[a];
            }
        }
        size_t p = 0;
        if (which & 1u) out[(p++) * nn + i] = sR;
        if (which & 2u) out[(p++) * nn + i] = sB;
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
    DomC &D = *(DomC *)(A.doms + dom);
    const size_t nn = (size_t)D.nx * D.ny;
    double sR = 0.0, sB = 0.0;
    for (size_t i = (size_t)b * MASS_THREADS + threadIdx.x; i < nn;
         i += (size_t)blocks_per_dom * MASS_THREADS) {
        const uint32_t m = A.mask[D.off + i];
        if (m & SELF_SOLID) continue;
        AT d[9], rR, rB;
        gather_global(A, D, (int)(i % D.nx), (int)(i / D.nx), m, d, rR, rB);
        sR += (double)rR;
        sB += (double)rB;
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

// ---------------------------------------------------------------- diagnostics (Sec. III)
// Max-reductions and sums in FP64 over the fluid nodes of a domain; DIAG_BLOCKS blocks per
// domain write partial results that a second kernel combines in a fixed order.
constexpr int DIAG_THREADS = 256;

__device__ __forceinline__ double block_max(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int k = DIAG_THREADS / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + k]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int k = DIAG_THREADS / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// |u|max (Eq. 46) and the largest change of a velocity component against a snapshot (Eq. 45)
template <class AT>
__global__ __launch_bounds__(DIAG_THREADS) void velocity_stats_kernel(
    const DomDev *doms, const uint16_t *mask, const AT *ux, const AT *uy, const AT *sx,
    const AT *sy, double *partials) {
    const int dom = blockIdx.x / DIAG_BLOCKS, b = blockIdx.x % DIAG_BLOCKS;
    const DomDev &D = doms[dom];
    const size_t nn = (size_t)D.nx * D.ny;
    double umax = 0.0, e1 = 0.0;
    for (size_t i = (size_t)b * DIAG_THREADS + threadIdx.x; i < nn; i += (size_t)DIAG_BLOCKS * DIAG_THREADS) {
        const size_t g = D.off + i;
        if (mask[g] & SELF_SOLID) continue;
        const double x = ux[g], y = uy[g];
        umax = fmax(umax, sqrt(x * x + y * y));
        if (sx) e1 = fmax(e1, fmax(fabs(x - (double)sx[g]), fabs(y - (double)sy[g])));
    }
    __shared__ double sh[DIAG_THREADS];
    umax = block_max(umax, sh);
    e1 = block_max(e1, sh);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = umax;
        partials[2 * blockIdx.x + 1] = e1;
    }
}

__global__ void max_final_kernel(const double *partials, int n_doms, double *out, int has_snap) {
    const int dom = blockIdx.x * blockDim.x + threadIdx.x;
    if (dom >= n_doms) return;
    double a = 0.0, e = 0.0;
    for (int b = 0; b < DIAG_BLOCKS; b++) {
        a = fmax(a, partials[2 * (dom * DIAG_BLOCKS + b)]);
        e = fmax(e, partials[2 * (dom * DIAG_BLOCKS + b) + 1]);
    }
    out[2 * dom] = a;
    out[2 * dom + 1] = has_snap ? e : __builtin_nan("");
}

template <class AT>
__global__ void velocity_copy_kernel(const DomDev *doms, int dom, const uint16_t *mask,
                                     const AT *ux, const AT *uy, double *ox, double *oy) {
    const DomDev &D = doms[dom];
    const size_t nn = (size_t)D.nx * D.ny;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nn; i += (size_t)gridDim.x * blockDim.x) {
        const size_t g = D.off + i;
        const bool fl = !(mask[g] & SELF_SOLID);
        if (ox) ox[i] = fl ? (double)ux[g] : 0.0;
        if (oy) oy[i] = fl ? (double)uy[g] : 0.0;
    }
}

// Colour masses inside and outside a region (the sums of Eq. 47)
template <class T>
__global__ __launch_bounds__(DIAG_THREADS) void region_mass_kernel(
    const StepArgs<T, typename Codec<T>::AT> A, int dom, const uint8_t *region, double *partials) {
    using AT = typename Codec<T>::AT;
    DomC &D = *(DomC *)(A.doms + dom);
    const size_t nn = (size_t)D.nx * D.ny;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (size_t i = blockIdx.x * (size_t)DIAG_THREADS + threadIdx.x; i < nn; i += (size_t)DIAG_BLOCKS * DIAG_THREADS) {
        const uint32_t m = A.mask[D.off + i];
        if (m & SELF_SOLID) continue;
        AT d[9], rR, rB;
        gather_global(A, D, (int)(i % D.nx), (int)(i / D.nx), m, d, rR, rB);
        const int k = region[i] ? 0 : 1;
        s[k] += (double)rR;
        s[2 + k] += (double)rB;
    }
    __shared__ double sh[DIAG_THREADS];
    for (int k = 0; k < 4; k++) {
        const double v = block_sum(s[k], sh);
        if (threadIdx.x == 0) partials[4 * blockIdx.x + k] = v;
    }
}

__global__ void sum4_final_kernel(const double *partials, double *out) {
    const int k = threadIdx.x;
    if (k >= 4) return;
    double v = 0.0;
    for (int b = 0; b < DIAG_BLOCKS; b++) v += partials[4 * b + k];
    out[k] = v;
}

// rho^N of node (x, y) from its gathered densities; 0 on solid nodes
template <class T>
__device__ double rho_n_at(const StepArgs<T, typename Codec<T>::AT> &A, DomC &D, int x, int y) {
    using AT = typename Codec<T>::AT;
    const uint32_t m = A.mask[D.off + (size_t)y * D.nx + x];
    if (m & SELF_SOLID) return 0.0;
    AT d[9], rR, rB;
    gather_global(A, D, x, y, m, d, rR, rB);
    return ((double)rR - (double)rB) / ((double)rR + (double)rB);
}

// One block per listed row: the first x with rho^N(x) > 0 >= rho^N(x + 1), interpolated
// linearly to x + rho^N(x) / (rho^N(x) - rho^N(x + 1))
template <class T>
__global__ __launch_bounds__(DIAG_THREADS) void crossing_kernel(
    const StepArgs<T, typename Codec<T>::AT> A, int dom, const int *rows, double *out) {
    DomC &D = *(DomC *)(A.doms + dom);
    const int y = rows[blockIdx.x];
    __shared__ int first;
    if (threadIdx.x == 0) first = D.nx;
    __syncthreads();
    if (y >= 0 && y < D.ny) {
        for (int x = threadIdx.x; x < D.nx - 1; x += DIAG_THREADS) {
            // early exit once some thread has found a crossing further left (an atomic read:
            // other threads lower the word concurrently; the result is read after the barrier)
            if (x >= __hip_atomic_load(&first, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
            if (rho_n_at(A, D, x, y) > 0.0 && rho_n_at(A, D, x + 1, y) <= 0.0) atomicMin(&first, x);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = __builtin_nan("");
        if (y >= 0 && y < D.ny && first < D.nx) {
            const double a = rho_n_at(A, D, first, y), b = rho_n_at(A, D, first + 1, y);
            r = first + a / (a - b);
        }
        out[blockIdx.x] = r;
    }
}

// ------------------------------------------------------------------- launchers
template <class T, bool WV>
static hipError_t step_t(const void *args, int n_items, int waves, int cols, int npl, hipStream_t s) {
    const auto &A = *static_cast<const StepArgs<T, typename Codec<T>::AT> *>(args);
    if constexpr (sizeof(typename Codec<T>::AT) == 4) {
        if (npl == 2) {
            if (waves == 8)
                hipLaunchKernelGGL((pair_kernel<T, 8, WV>), dim3(n_items), dim3(TILE_LANES * 8), 0, s, A);
            else
                hipLaunchKernelGGL((pair_kernel<T, 4, WV>), dim3(n_items), dim3(TILE_LANES * 4), 0, s, A);
            return hipGetLastError();
        }
    }
    if (npl != 1) return hipErrorInvalidValue;
    if (cols == 2)
        hipLaunchKernelGGL((step_kernel<T, 4, 2, WV>), dim3(n_items), dim3(TILE_LANES * 8), 0, s, A);
    else if (waves == 8)
        hipLaunchKernelGGL((step_kernel<T, 8, 1, WV>), dim3(n_items), dim3(TILE_LANES * 8), 0, s, A);
    else
        hipLaunchKernelGGL((step_kernel<T, 4, 1, WV>), dim3(n_items), dim3(TILE_LANES * 4), 0, s, A);
    return hipGetLastError();
}

template <class T>
static hipError_t step_v(const void *args, int n_items, int waves, int cols, int npl, bool variants,
                         hipStream_t s) {
    return variants ? step_t<T, true>(args, n_items, waves, cols, npl, s)
                    : step_t<T, false>(args, n_items, waves, cols, npl, s);
}

hipError_t launch_step(int storage, const void *args, int n_items, int waves, int cols, int npl,
                       bool variants, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    switch (storage) {
        case 0: return step_v<double>(args, n_items, waves, cols, npl, variants, s);
        case 1: return step_v<float>(args, n_items, waves, cols, npl, variants, s);
        case 2: return step_v<__half>(args, n_items, waves, cols, npl, variants, s);
        case 3: return step_v<C16>(args, n_items, waves, cols, npl, variants, s);
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
        case 3: return read_t<C16>(args, dom, nx, ny, which, out, s);
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
        case 3: return mass_t<C16>(args, n_doms, partials, bpd, out, s);
    }
    return hipErrorInvalidValue;
}

template <class T>
static const StepArgs<T, typename Codec<T>::AT> &args_of(const void *a) {
    return *static_cast<const StepArgs<T, typename Codec<T>::AT> *>(a);
}

template <class T>
static hipError_t velocity_stats_t(const void *args, int n_doms, const void *u, const void *snap,
                                   double *partials, double *out, hipStream_t s) {
    using AT = typename Codec<T>::AT;
    const auto &A = args_of<T>(args);
    const size_t stride = A.c_plane_bytes / sizeof(AT);
    const AT *ux = static_cast<const AT *>(u), *sx = static_cast<const AT *>(snap);
    hipLaunchKernelGGL(velocity_stats_kernel<AT>, dim3(n_doms * DIAG_BLOCKS), dim3(DIAG_THREADS), 0, s,
                       A.doms, A.mask, ux, ux + stride, sx, sx ? sx + stride : nullptr, partials);
    hipLaunchKernelGGL(max_final_kernel, dim3((n_doms + 63) / 64), dim3(64), 0, s, partials, n_doms,
                       out, snap != nullptr);
    return hipGetLastError();
}

template <class T>
static hipError_t velocity_copy_t(const void *args, int dom, const void *u, double *ox, double *oy,
                                  hipStream_t s) {
    using AT = typename Codec<T>::AT;
    const auto &A = args_of<T>(args);
    const size_t stride = A.c_plane_bytes / sizeof(AT);
    const AT *ux = static_cast<const AT *>(u);
    hipLaunchKernelGGL(velocity_copy_kernel<AT>, dim3(1024), dim3(256), 0, s, A.doms, dom, A.mask, ux,
                       ux + stride, ox, oy);
    return hipGetLastError();
}

template <class T>
static hipError_t region_mass_t(const void *args, int dom, const uint8_t *region, double *partials,
                                double *out, hipStream_t s) {
    hipLaunchKernelGGL(region_mass_kernel<T>, dim3(DIAG_BLOCKS), dim3(DIAG_THREADS), 0, s, args_of<T>(args),
                       dom, region, partials);
    hipLaunchKernelGGL(sum4_final_kernel, dim3(1), dim3(64), 0, s, partials, out);
    return hipGetLastError();
}

template <class T>
static hipError_t crossings_t(const void *args, int dom, const int *rows, int n_rows, double *out,
                              hipStream_t s) {
    hipLaunchKernelGGL(crossing_kernel<T>, dim3(n_rows), dim3(DIAG_THREADS), 0, s, args_of<T>(args), dom,
                       rows, out);
    return hipGetLastError();
}

hipError_t launch_velocity_stats(int storage, const void *args, int n_doms, const void *u,
                                 const void *snap, double *partials, double *out, hipStream_t s) {
#define CALL(T) velocity_stats_t<T>(args, n_doms, u, snap, partials, out, s)
    switch (storage) {
        case 0: return CALL(double);
        case 1: return CALL(float);
        case 2: return CALL(__half);
        case 3: return CALL(C16);
    }
#undef CALL
    return hipErrorInvalidValue;
}

hipError_t launch_velocity_copy(int storage, const void *args, int dom, const void *u, double *ox,
                                double *oy, hipStream_t s) {
#define CALL(T) velocity_copy_t<T>(args, dom, u, ox, oy, s)
    switch (storage) {
        case 0: return CALL(double);
        case 1: return CALL(float);
        case 2: return CALL(__half);
        case 3: return CALL(C16);
    }
#undef CALL
    return hipErrorInvalidValue;
}

hipError_t launch_region_mass(int storage, const void *args, int dom, const uint8_t *region,
                              double *partials, double *out, hipStream_t s) {
#define CALL(T) region_mass_t<T>(args, dom, region, partials, out, s)
    switch (storage) {
        case 0: return CALL(double);
        case 1: return CALL(float);
        case 2: return CALL(__half);
        case 3: return CALL(C16);
    }
#undef CALL
    return hipErrorInvalidValue;
}

hipError_t launch_crossings(int storage, const void *args, int dom, const int *rows, int n_rows,
                            double *out, hipStream_t s) {
#define CALL(T) crossings_t<T>(args, dom, rows, n_rows, out, s)
    switch (storage) {
        case 0: return CALL(double);
        case 1: return CALL(float);
        case 2: return CALL(__half);
        case 3: return CALL(C16);
    }
#undef CALL
    return hipErrorInvalidValue;
}

// ------------------------------------------ device-resident staging of the no-alloc crossings
// Row list (NOALLOC_ROWS ints) followed by the results (NOALLOC_ROWS doubles) of
// lbm_diag_crossings_noalloc.  One copy per GPU, kept until the process ends.  In host code the
// name `scratch` is only a host-side stand-in for the symbol: kernels get the device address
// that hipGetSymbolAddress returns for the current device (noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        // once per device, with that device current (the caller's responsibility)
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

hipError_t launch_crossings_noalloc(int storage, const void *args, int dom, void *scratch_dev,
                                    int n_rows, hipStream_t s) {
    const int *rows = static_cast<const int *>(scratch_dev);
    double *out = reinterpret_cast<double *>(static_cast<char *>(scratch_dev) + NOALLOC_OUT_OFFSET);
    return launch_crossings(storage, args, dom, rows, n_rows, out, s);
}

}  // namespace lbmcg
