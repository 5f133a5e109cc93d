// Internal layout shared by the kernels and the host runtime of lbmcg.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbmcg {

// Per-node class word.  Bits 0..7: the stencil neighbour in direction a = 1..8 is solid
// (bit a-1).  Neighbours wrap periodically in y, and in x unless the x axis is open, where
// they are clamped to the edge column.
constexpr uint32_t SELF_SOLID = 1u << 8;
constexpr uint32_t FLUID_BND = 1u << 9;   // fluid node with a solid neighbour
constexpr uint32_t SOLID_BND = 1u << 10;  // solid node with a fluid neighbour

constexpr int TILE_LANES = 64;     // columns per tile row (one wavefront)
constexpr int HALO = 5;            // halo rows per side: the step's dependency radius next to
                                   // walls is 4, plus one row for the colour-state stencil
// Halo columns per side of the one-column-per-lane step kernel.  With FP64 arithmetic the
// colour-state column beyond the radius is a lane of the window (5); with FP32 arithmetic it is
// loaded into two extra LDS columns instead, so every lane gathers and the halo is the radius
// (4): 56 output columns per wavefront instead of 54.
constexpr int HALO_X64 = 5, HALO_X32 = 4;
inline int halo_x(int storage) { return storage == 0 ? HALO_X64 : HALO_X32; }
// Output columns of a tile: `cols` wavefronts side by side with one column per lane, or one
// wavefront with two columns per lane (npl = 2: 128 columns, halo 6).  The FP64 storage uses
// the one-column kernel only.
inline int tile_out(int cols, int npl, int storage) {
    return npl == 2 ? 2 * TILE_LANES - 12 : TILE_LANES * cols - 2 * halo_x(storage);
}

// Per-domain parameters in one arithmetic type, with the constant factors of the collision
// precomputed: ke = 6 (1 - s_e / 2), keps = 6 (1 - s_eps / 2), kq = 1 - s_q / 2 (the forcing
// terms of Eq. 8 for e, epsilon and q).
template <class AT>
struct DomPar {
    AT rho0, eps, inv2nu_r, inv2nu_b, half_sigma, beta, cos_t, sin_t;
    AT s_e, s_eps, s_q, ke, keps, kq, outlet_u, pad;
};

// Wetting variants (same values as the LBM_WET_* flags of the interface).
constexpr int WET_SCHEME_B = 1;         // Eq. 48 for grad n on outermost fluid nodes
constexpr int WET_SURFACE_ENERGY = 2;   // rho^N = cos(theta) on outermost solid nodes

struct DomDev {
    long long off;       // first node of the domain in every node plane
    int nx, ny;
    int open_x, wetting;
    long long io_off;    // first row of the domain in the inlet / outlet row arrays
    DomPar<double> d;    // parameters for FP64 arithmetic
    DomPar<float> f;     // the same, rounded once, for FP32 arithmetic
};

// FP16 storage scale of direction a (the device codec uses the same constants).
inline float fp16_scale(int a) { return a == 0 ? 512.0f : (a < 5 ? 2048.0f : 8192.0f); }

// 16-bit storage with one more significand bit than binary16: sign, 4-bit exponent (bias 7),
// 11-bit fraction, subnormals at exponent 0.  A population deviation d of direction a is
// stored as d * fp16_scale(a), so that the format covers |d| < 2.25 w_a rho0 (larger values
// saturate) with a relative rounding error below 2^-12.
struct C16 {
    uint16_t bits;
};

struct WorkItem {
    int dom, x0, y0, y1;
};

// Pointers of one step.  f* are 9 planes of `plane` elements (direction-major), c / vx / vy
// one plane each (colour state of the node's last collision), hist is the outlet history:
// [row][3] deviations of f_3, f_6, f_7 at the outlet column.
template <class T, class AT>
struct StepArgs {
    const DomDev *doms;
    const WorkItem *items;
    int n_items;
    int own;  // state is a node-local snapshot: f at its node, c = red fraction, v unused
    const T *fin;
    const AT *cin, *vxin, *vyin;
    T *fout;
    AT *cout, *vxout, *vyout;
    const AT *hist_in;
    AT *hist_out;
    const uint16_t *mask;
    const AT *ns;  // wall normal (x, y) per node, interleaved
    const AT *inlet;
    size_t plane;
    int *flag;
    // Byte extents for the step kernel's buffer accesses (each below 2^31, checked on the
    // host): one population plane, the 9 population planes, one colour-state plane (c, vx and
    // vy planes follow each other at this stride), and the interleaved wall normals.
    uint32_t f_plane_bytes, f_set_bytes, c_plane_bytes, ns_bytes;
    // Diagnostic launch (diag != 0): the state is read as in a step but nothing is written
    // back (no populations, colour state or outlet history); instead the velocity of Eq. 17
    // (with the half-force term) of every fluid node goes to u_out, u_x then u_y, planes
    // c_plane_bytes apart (through the colour-state stores of the step).
    AT *u_out;
    int diag;
    // Contact-line list of a diagnostic launch (cl_count == nullptr: none): every outermost
    // fluid node of domain cl_dom with |grad rho^N| > eps (before the correction of Eqs. 30-36)
    // adds one to *cl_count and, while there is room, its index y * nx + x to cl_list (cl_cap
    // entries, in no particular order).
    int32_t *cl_list;
    int *cl_count;
    int cl_cap, cl_dom;
};

// Launchers (lbm_kernels.hip).  storage: 0 f64, 1 f32, 2 f16, 3 c16.
// waves x cols wavefronts per block: (4, 1), (8, 1) or (4, 2); a tile is 64 cols columns wide.
// npl: node columns per lane, 1, or 2 (the pair kernel: FP32-arithmetic storages, cols = 1,
// every domain of even width; the tile is then 128 columns wide).
// variants: some domain has nonzero wetting flags (selects the kernel that tests them).
hipError_t launch_step(int storage, const void *args, int n_items, int waves, int cols, int npl,
                       bool variants, hipStream_t s);
hipError_t launch_read(int storage, const void *args, int dom, int nx, int ny, uint32_t which,
                       double *out, hipStream_t s);
hipError_t launch_mass(int storage, const void *args, int n_doms, const int *dom_nodes_begin,
                       double *partials, int n_blocks_per_dom, double *out, hipStream_t s);

// Diagnostics (lbm_kernels.hip).
constexpr int DIAG_BLOCKS = 64;     // blocks per domain of the diagnostic reductions
constexpr int DIAG_MAX_ROWS = 4096;  // rows per lbm_diag_crossings call
// Per domain: |u|max over fluid nodes, and max(|u_x - s_x|, |u_y - s_y|) against the snapshot.
hipError_t launch_velocity_stats(int storage, const void *args, int n_doms, const void *u,
                                 const void *snap, double *partials, double *out, hipStream_t s);
// u_x, u_y of one domain as FP64 planes (solid nodes 0); either output may be NULL.
hipError_t launch_velocity_copy(int storage, const void *args, int dom, const void *u,
                                double *ox, double *oy, hipStream_t s);
// FP64 {sum rho_R, sum rho_B} over fluid nodes with region != 0, then region == 0.
hipError_t launch_region_mass(int storage, const void *args, int dom, const uint8_t *region,
                              double *partials, double *out, hipStream_t s);
// First x of each listed row where rho^N goes from > 0 to <= 0 (interpolated), NaN if none.
hipError_t launch_crossings(int storage, const void *args, int dom, const int *rows, int n_rows,
                            double *out, hipStream_t s);

// Staging of lbm_diag_crossings_noalloc in a static device array (lbm_kernels.hip): up to
// NOALLOC_ROWS row indices, then as many FP64 results at byte NOALLOC_OUT_OFFSET.
constexpr int NOALLOC_ROWS = 4096;
constexpr size_t NOALLOC_OUT_OFFSET = NOALLOC_ROWS * sizeof(int);
constexpr size_t NOALLOC_SCRATCH_BYTES = NOALLOC_OUT_OFFSET + NOALLOC_ROWS * sizeof(double);
// Device address of that array on `device`, which must be the current device; looked up once
// per device with hipGetSymbolAddress and cached.
hipError_t noalloc_scratch(int device, void **out);
// crossing_kernel with rows and results in the array at scratch_dev (noalloc_scratch's address).
hipError_t launch_crossings_noalloc(int storage, const void *args, int dom, void *scratch_dev,
                                    int n_rows, hipStream_t s);

}  // namespace lbmcg
