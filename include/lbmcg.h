/*
 * lbmcg: MI355X (gfx950) library for the two-colour D2Q9 lattice Boltzmann time step with the
 * improved geometric wetting boundary of Yu, Liu, Zhang and Liang (arXiv:1707.00198).
 *
 * One call of lbm_step advances every domain of a context by the method of Sec. II:
 * MRT collision with the CSF interfacial force and Guo forcing (Eqs. 1-13, 16-18),
 * Latva-Kokko/Rothman recolouring (Eq. 14), streaming with half-way bounce-back (Eq. 15),
 * and the wetting boundary of Sec. II C: virtual colour values on the outermost solid nodes
 * (Eq. 29), the wall normal from the eighth-order stencil (Eqs. 32-33) or from the caller,
 * the contact-angle rotation and selection of the colour-gradient direction (Eqs. 30-36),
 * and virtual interface normals on the outermost solid nodes (Eq. 29 applied to n, which
 * imposes the zero interface force of Eqs. 19-27 and 37-44).
 *
 * Conventions shared by every entry point:
 *  - A domain is an nx * ny lattice that includes its solid nodes; node (x, y) is element
 *    y * nx + x of every per-node host array.  Lattice directions follow the paper:
 *    e0 = (0,0), e1 = (1,0), e2 = (0,1), e3 = (-1,0), e4 = (0,-1), e5 = (1,1), e6 = (-1,1),
 *    e7 = (-1,-1), e8 = (1,-1).
 *  - y is periodic; walls are solid nodes of the mask.  x is periodic, or (open_x) has a
 *    Zou-He velocity inlet at x = 0 and a convective outlet at x = nx - 1.
 *  - All device pointers belong to the caller and stay owned by the caller; the library
 *    borrows the state and scratch buffers from lbm_create until lbm_destroy.  The library
 *    itself owns only the context object, host-side tables and, once lbm_set_graph turns
 *    them on, its step graphs and the private stream they are captured on; it allocates no
 *    device memory.
 *  - Every call returns an lbm_status; nothing throws across this interface.  The text of
 *    the last error on the calling thread is returned by lbm_last_error.
 *  - Work is enqueued on the HIP stream given to lbm_create and is asynchronous unless the
 *    entry point says otherwise.
 *  - A context is used by one thread at a time (calls change its step parity, schedule and
 *    graphs); separate contexts may be driven from separate threads.
 */
#ifndef LBMCG_H
#define LBMCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,      /* invalid argument or parameter (detected before any device work) */
    LBM_ENOMEM = -2,      /* caller buffer too small */
    LBM_EDEVICE = -3,     /* a HIP call failed */
    LBM_ENONFINITE = -4,  /* a non-finite density or velocity appeared on the device */
    LBM_ESTATE = -5       /* call not valid in the context's current state */
} lbm_status;

/* Population storage.  Arithmetic is FP64 for LBM_STORE_F64 and FP32 otherwise.  Populations
 * are stored as deviations f_alpha - w_alpha * rho0.  The 16-bit storages multiply them by a
 * power-of-two scale per direction (2^9 rest, 2^11 axis, 2^13 diagonal): LBM_STORE_F16 stores
 * binary16, LBM_STORE_C16 a format with one more significand bit (sign, 4-bit exponent with
 * bias 7, 11-bit fraction, subnormals; saturating beyond |deviation| = 2.25 w_alpha rho0).  The
 * step kernels round both 16-bit formats stochastically (each value goes to one of its two
 * neighbouring codes, up with a probability equal to the dropped fraction; error below one
 * unit, 2^-10 relative for binary16 and 2^-11 for LBM_STORE_C16, with no systematic part; the
 * random bits are a hash of the node's position in its domain and of its state, so a run is
 * reproducible and a domain gives the same results alone or in any batch); the initial upload
 * rounds to nearest.  Colour state is FP64 / FP32.
 * Accuracy against FP64 storage on the 16384 x 512 displacement channel after 30000 steps:
 * finger length within 0.12 % (FP32), 0.001 % (LBM_STORE_C16) and 0.21 % (LBM_STORE_F16), tip
 * velocity within 0.005 %.  Capillary filling (Eq. 49) is where the 16-bit formats differ:
 * meniscus travel within 0.8 % (LBM_STORE_C16) and 1.0-1.3 % (LBM_STORE_F16), so runs held to
 * a 1 % bar should use LBM_STORE_C16. */
typedef enum {
    LBM_STORE_F64 = 0,
    LBM_STORE_F32 = 1,
    LBM_STORE_F16 = 2,
    LBM_STORE_C16 = 3
} lbm_storage;

/* Wetting variants of Sec. III A (flags of lbm_domain_desc.wetting; 0 is the paper's model:
 * virtual rho^N and virtual normals on outermost solid nodes by Eq. 29, the colour gradient
 * on outermost fluid nodes corrected by Eqs. 30-36).
 *  LBM_WET_SCHEME_B: scheme (b) of Sec. III A 2.  No virtual normals; on outermost fluid nodes
 *    the derivatives of n in the curvature (Eq. 13) come from the one-sided mean of Eq. 48
 *    over the directions whose neighbour is fluid.
 *  LBM_WET_SURFACE_ENERGY: the surface-energy rule of Sec. III A 1.  The virtual rho^N on
 *    outermost solid nodes is cos(theta) instead of Eq. 29, and the gradient is not corrected.
 * The flags combine; the surface-energy model compared in Fig. 2, which has no
 * zero-interface-force condition, is both together. */
#define LBM_WET_SCHEME_B 1
#define LBM_WET_SURFACE_ENERGY 2

/* One domain.  Host pointers are read during lbm_create only. */
typedef struct {
    int32_t nx, ny;           /* lattice extent including solid nodes; nx >= 2 if open_x */
    int32_t open_x;           /* 0: periodic x; 1: velocity inlet at x = 0, outlet at nx-1 */
    int32_t wetting;          /* LBM_WET_* flags (0: the paper's model); other bits invalid */
    const uint8_t *solid;     /* nx*ny, nonzero = solid (required) */
    const double *ns;         /* optional nx*ny*2 wall normal pointing into the solid,
                                 used on outermost fluid nodes; NULL = eighth-order stencil */
    const double *inlet_ux;   /* ny inlet velocities (required if open_x, else ignored) */
    const double *rho_r0;     /* nx*ny initial red density (fluid nodes) */
    const double *rho_b0;     /* nx*ny initial blue density; rho_r0 + rho_b0 > 0 on fluid */
    double nu_r, nu_b;        /* kinematic viscosities (> 0), Eqs. 5 and 18 */
    double sigma;             /* interfacial tension coefficient (>= 0), Eq. 10 */
    double beta;              /* recolouring segregation parameter in [0, 1], Eq. 14 */
    double theta_deg;         /* prescribed contact angle in [0, 180], measured in red */
    double s_e, s_eps, s_q;   /* relaxation rates of e, epsilon, q in (0, 2), Eq. 6 */
    double rho0;              /* reference density (> 0) of the population deviations */
    double eps;               /* |grad rho^N| threshold (> 0) below which n = 0 */
    double outlet_u;          /* convective outlet velocity (>= 0) */
} lbm_domain_desc;

/* Bytes of device memory the caller must provide for `n` domains stored as `storage`:
 * `state_bytes` (populations, colour state, open-boundary history; rewritten every step)
 * and `scratch_bytes` (node classes, wall normals, tables; written once by lbm_create).
 * Returns LBM_EINVAL for an invalid descriptor. */
int lbm_query_bytes(const lbm_domain_desc *domains, int n, int storage, size_t *state_bytes,
                    size_t *scratch_bytes);

/* Validate, classify nodes (fluid, outermost fluid, outermost solid, solid), compute wall
 * normals, build the tile schedule and upload everything plus the initial state
 * (f_alpha = rho_k w_alpha, u = 0) into `state_dev` / `scratch_dev` (device pointers of at
 * least the queried sizes, 256-byte aligned) of the device current during the call, which
 * becomes the context's device.  `hip_stream` is a hipStream_t of that device (NULL = the
 * default stream).  Blocks until the upload has finished.  On success *out owns a context.
 * LBM_EINVAL for an invalid descriptor, NULL or misaligned buffers, or a batch beyond one
 * context's limit (2^31 bytes for the nine population planes and for the three colour-state
 * planes); LBM_ENOMEM if a buffer is smaller than lbm_query_bytes reports. */
int lbm_create(const lbm_domain_desc *domains, int n, int storage, void *state_dev,
               size_t state_bytes, void *scratch_dev, size_t scratch_bytes, void *hip_stream,
               lbm_ctx **out);

/* Host-only: node classes and wall normals the library derives for one domain, without any
 * device work.  classes_out (nx*ny, may be NULL): 0 fluid, 1 outermost fluid (a fluid node with
 * a solid D2Q9 neighbour), 2 outermost solid (a solid node with a fluid neighbour), 3 other
 * solid.  ns_out (nx*ny*2, may be NULL): the wall normal used on outermost fluid nodes
 * (Eqs. 32-33 or the caller's analytic normal, unit length, into the solid), 0 elsewhere. */
int lbm_classify(const lbm_domain_desc *domain, uint8_t *classes_out, double *ns_out);

/* Enqueue n_steps time steps of every domain on the context's stream (asynchronous).  With
 * step graphs on (lbm_set_graph), runs of steps go out as replays of an instantiated HIP graph
 * of that many step launches; results are the same bit for bit either way.  LBM_EINVAL for a
 * negative count; LBM_EDEVICE if a launch (or the first capture of a graph) fails. */
int lbm_step(lbm_ctx *ctx, int64_t n_steps);

/* Step graphs: `launches` step launches (0 = off, the default, else even, 2..1024) are
 * captured once per starting buffer parity on a private stream of the library and replayed on
 * the context's stream, one graph launch per `launches` steps.  The initial state of a context
 * (node-local, not yet streamed; also after lbm_load_state of such a state) first takes one
 * direct step, and a remainder shorter than a graph is launched step by step.  The graphs are
 * rebuilt after lbm_set_tile and lbm_autotune.  Both graphs are captured, instantiated and
 * uploaded to the device by this call (rebuilt ones at their first replay).  Synchronises the
 * stream.  LBM_EINVAL for an odd or out-of-range count; LBM_EDEVICE if a capture fails. */
int lbm_set_graph(lbm_ctx *ctx, int launches);

/* Autotuner of the step's tile shape on this context's own batch: times every provided shape,
 * chunk_rows in {8, 12, 16, 24, 32, 48, 64} (shapes that cut no domain differently are timed
 * once) x (waves, cols, cols_per_lane) in {(4, 1, 1), (8, 1, 1), (4, 2, 1)}, plus (4, 1, 2) and
 * (8, 1, 2) where lbm_set_tile allows two columns per lane, with `steps` (1..100000) timed steps
 * after one untimed step each, re-times the three fastest and keeps the fastest (as
 * lbm_set_tile).  The trials run real steps, so the state is first saved to `save_dev`
 * (caller-owned device buffer of lbm_state_size bytes) and restored afterwards: the state, the
 * step count and the non-finite flag are as before the call.  If `out_host` is not NULL it
 * receives (chunk_rows, waves, cols, milliseconds per step, cols_per_lane) of the choice.
 * Synchronises the stream.  On LBM_EDEVICE the state is undefined. */
int lbm_autotune(lbm_ctx *ctx, int steps, void *save_dev, double *out_host);

/* Field selection bits for lbm_read_fields. */
#define LBM_FIELD_RHO_R 1u   /* red density, Eq. 16 (one plane) */
#define LBM_FIELD_RHO_B 2u   /* blue density (one plane) */
#define LBM_FIELD_POPS 4u    /* post-streaming populations f_{alpha,k}: 18 planes, colour-major
                                (red alpha 0..8, then blue alpha 0..8) */
#define LBM_FIELD_UX 8u      /* velocity u_x of Eq. 17 (with the half-force term) that the next
                                collision uses (one plane; needs lbm_diag_attach) */
#define LBM_FIELD_UY 16u     /* velocity u_y, likewise */

/* Decode domain `domain`'s current state to FP64 into `out_dev` (device pointer, capacity
 * `out_count` doubles): one nx*ny plane per selected quantity, in bit order; solid nodes
 * read 0.  Enqueued on the context's stream.  LBM_ENOMEM if out_count is too small.  The
 * velocity planes are computed by a diagnostic launch of the step (no state is changed) and
 * need an attached diagnostics buffer (LBM_ESTATE otherwise).  LBM_EINVAL for an unknown
 * domain, an empty or unknown field selection, or a NULL output. */
int lbm_read_fields(lbm_ctx *ctx, int domain, uint32_t which, double *out_dev,
                    size_t out_count);

/* Per-domain FP64 sums over fluid nodes of rho_R and rho_B into out_host[2*d], [2*d + 1].
 * Synchronises the stream.  Returns LBM_ENONFINITE if a step has produced a non-finite
 * density or velocity since the context was created. */
int lbm_mass(lbm_ctx *ctx, double *out_host);

/* Number of time steps taken so far. */
int64_t lbm_steps_taken(const lbm_ctx *ctx);

/* Tile shape of the fused step: `chunk_rows` rows of a strip per work item (multiple of 4,
 * >= 8; 0 = built-in choice), `waves` tile rows advanced per iteration (4 or 8; 0 = built-in),
 * `cols` wavefronts side by side in a tile row and `cols_per_lane` node columns per lane:
 *   cols 1, cols_per_lane 1: 64-column tiles with 56 output columns (54 for LBM_STORE_F64);
 *   cols 2, cols_per_lane 1: 128-column tiles with 120 output columns (118 for LBM_STORE_F64;
 *     8 x 2 not provided);
 *   cols 1, cols_per_lane 2: 128-column tiles with 116 output columns, each lane updating two
 *     adjacent nodes; only for the FP32-arithmetic storages and batches whose domains all have an
 *     even nx (never the built-in choice; lbm_autotune weighs it).
 * 0 selects the built-in value.  Rebuilds the schedule.  Every shape computes the same method
 * with the same per-node arithmetic (FP64: the same bits; FP32 arithmetic: each shape is checked
 * against the FP64 oracle to the storage's rounding).  Synchronises the stream.  LBM_EINVAL for a
 * shape outside these. */
int lbm_set_tile(lbm_ctx *ctx, int chunk_rows, int waves, int cols, int cols_per_lane);

/* The tile shape in use (the built-in choice, lbm_set_tile's or lbm_autotune's): shape_out
 * (host, 5 ints) receives chunk_rows, waves, cols, the number of work items (blocks per step
 * launch) and cols_per_lane.  Host-only.  LBM_EINVAL for a NULL argument. */
int lbm_get_tile(const lbm_ctx *ctx, int *shape_out);

/* Checkpoint: copy the complete mutable state (state buffer contents plus step parity, count
 * and snapshot mode) to `dst_dev` (device, lbm_state_size bytes) or restore it from `src_dev`.
 * Both synchronise the stream.  `src_dev` must come from lbm_save_state of a context with the
 * same domains and storage; lbm_load_state returns LBM_ESTATE if it finds no saved-state header
 * at the end of the buffer. */
size_t lbm_state_size(const lbm_ctx *ctx);
int lbm_save_state(lbm_ctx *ctx, void *dst_dev);
int lbm_load_state(lbm_ctx *ctx, const void *src_dev);

/* Diagnostics of Sec. III (Eqs. 45-47), computed on the device from the current state.
 * They need a caller-owned device buffer of lbm_diag_bytes bytes (256-byte aligned), handed
 * over with lbm_diag_attach (NULL detaches); the library borrows it until it is detached or the
 * context destroyed.  Each call synchronises the context's stream. */
size_t lbm_diag_bytes(const lbm_ctx *ctx);
int lbm_diag_attach(lbm_ctx *ctx, void *diag_dev, size_t bytes);

/* Velocity statistics of every domain, without advancing the state: out_host[2*d] = |u|max
 * (Eq. 46) over the fluid nodes of domain d, with u of Eq. 17 including the half-force term;
 * out_host[2*d + 1] = max over fluid nodes of max(|u_x - u_x^s|, |u_y - u_y^s|) against the
 * snapshot u^s (Eq. 45 when the snapshot was taken 500 steps earlier), NaN if no snapshot has
 * been taken since lbm_diag_attach.  If `snapshot` is nonzero the current velocity becomes the
 * snapshot afterwards.  LBM_ENONFINITE as lbm_mass. */
int lbm_diag_velocity(lbm_ctx *ctx, int snapshot, double *out_host);

/* FP64 colour masses of domain `domain` split by a region (the sums of Eq. 47): region_dev is a
 * device array of nx*ny bytes (nonzero = inside); out_host[0..3] = sum of rho_R inside, rho_R
 * outside, rho_B inside, rho_B outside, over fluid nodes. */
int lbm_diag_region_mass(lbm_ctx *ctx, int domain, const uint8_t *region_dev, double *out_host);

/* Interface positions along rows (contact line and finger tip of Sec. III): for each of the
 * n_rows (1..4096) rows in rows_host, the first x, scanning from x = 0, with rho^N(x) > 0 >=
 * rho^N(x + 1), interpolated linearly to x + rho^N(x) / (rho^N(x) - rho^N(x + 1)); NaN if the
 * row has none.  rho^N of Eq. 12 from the current densities, 0 on solid nodes. */
int lbm_diag_crossings(lbm_ctx *ctx, int domain, const int32_t *rows_host, int n_rows,
                       double *out_host);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): lbm_diag_crossings without a diagnostics buffer.  Same
 * arguments and results, but the row list and the results are staged in a static device array of
 * the library (one per GPU, LBM_NOALLOC_MAX_ROWS rows, 48 KiB, held until the process ends) and
 * copied from / to the caller's plain host arrays; nothing is allocated, no diagnostics buffer is
 * needed.  The array is looked up once per device by lbm_create (on the device current there).
 * Synchronises the context's stream.  LBM_EINVAL for n_rows outside [1, LBM_NOALLOC_MAX_ROWS] or a
 * row outside the domain, before any device work.  Every call on one GPU, from any context or
 * thread, shares that GPU's array: calls that overlap in time on one GPU race. */
#define LBM_NOALLOC_MAX_ROWS 4096
int lbm_diag_crossings_noalloc(lbm_ctx *ctx, int domain, const int32_t *rows_host, int n_rows,
                               double *out_host);

/* The dynamic contact-line list (the part of the outermost fluid nodes where the wetting
 * condition of Sec. II C acts): the outermost fluid nodes of `domain` whose colour gradient of
 * the current state (Eq. 28 with the virtual values, before the correction of Eqs. 30-36) has
 * |grad rho^N| > eps.  Pure-phase wall regions, where the gradient vanishes, are not listed.
 * Computed on the device by a diagnostic launch (no state is written).  Sets *count to the
 * number of such nodes and writes their indices y * nx + x in ascending order to out_host
 * (host array of `cap` entries); LBM_ENOMEM, with *count set and out_host untouched, if
 * *count > cap.  Needs an attached diagnostics buffer. */
int lbm_diag_contact_line(lbm_ctx *ctx, int domain, int32_t *out_host, int cap, int *count);

/* Message of the last failed call on this thread ("" if none). */
const char *lbm_last_error(void);

/* Release the context (does not free the caller's buffers).  Synchronises the stream. */
void lbm_destroy(lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBMCG_H */
