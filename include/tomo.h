/*
 * tomo.h -- C ABI of libtomo, a gfx950 (MI355X) implementation of the
 * line-of-sight projector of TomograPy (Barbey, Guennou & Auchere, Solar
 * Physics), its exact transpose, and the conjugate-gradient inversion of the
 * paper's regularised least-squares criterion.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Voxel cube (Sec. "Single Spacecraft Static Tomography"): nx*ny*nz
 *   identical rectangular voxels filling the box [box_min, box_max]; FP32,
 *   x fastest: index = (k*ny + j)*nx + i.  A cube argument holding nframes
 *   time frames is nframes such volumes back to back (the block-diagonal
 *   operator of Eq. srt_t).  Voxels are half-open [lo + k D, lo + (k+1) D).
 * - Images (Eq. srt): FP32, the views concatenated in order, each view
 *   [nrow][ncol] with the column fastest.
 * - Line of sight through pixel (col, row) of a view: the half-line
 *   obs + t d, t >= 0, with d = w + (col - crpix0) cdelt0 u
 *   + (row - crpix1) cdelt1 v (gnomonic / TAN projection; the paper defines
 *   observer and projector through WCS keywords, Sec. "Instrument
 *   Independence").  w, u, v must be orthonormal.  Pixel centres sit at
 *   integer 0-based indices.  Lengths are in box units.
 * - Projection (Eq. lo): image value = sum over the voxels the line crosses
 *   of (length inside the voxel) * (voxel value), computed with Siddon's
 *   method: the ray's crossings of the x, y and z voxel planes are merged in
 *   order (simultaneous crossings taken as one).  The transpose scatters the
 *   same lengths, so the two are exact adjoints of one another.
 * - Masks (Sec. "Performance"): data_mask[ray] == 0 removes a pixel (its
 *   row of P is zero, and it is neither projected nor back-projected);
 *   map_mask[voxel] == 0 removes a voxel from the unknowns, so the operator
 *   is P M with M the 0/1 diagonal of the map mask.
 *
 * Memory and streams
 * ------------------
 * Cube, image and mask arrays are caller-owned DEVICE pointers (contiguous).
 * tomo_view arrays and all structs are HOST memory.  A stream argument is a
 * hipStream_t (NULL = the default stream); work is enqueued asynchronously
 * on it unless a call says otherwise, and kernel faults surface at the next
 * synchronising call.  The library caches device copies of view tables,
 * keyed by the geometry's contents: the first call with a new geometry
 * allocates and uploads synchronously, so make that call before any stream
 * capture.  tomo_release_cache() frees the cache.
 *
 * Errors
 * ------
 * Every call returns TOMO_OK (0) or a negative tomo_status; nothing aborts
 * or throws across the ABI.  Invalid arguments are rejected before any GPU
 * work is enqueued.  tomo_last_error() returns a text for the last failure
 * on the calling thread.
 */
#ifndef TOMO_H
#define TOMO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *tomo_stream; /* hipStream_t */

typedef enum tomo_status {
    TOMO_OK = 0,
    TOMO_EINVAL = -1,      /* bad sizes, bounds, frame, NULL pointer, ...      */
    TOMO_EHIP = -2,        /* a HIP runtime call failed                         */
    TOMO_ENONFINITE = -3,  /* a solver scalar became NaN or infinite            */
    TOMO_ENOCONV = -4,     /* max_iter reached before rtol (report only)        */
    TOMO_ENOMEM = -5,      /* device or host allocation failed                  */
    TOMO_EUNSUPPORTED = -6 /* option not supported with these arguments         */
} tomo_status;

typedef struct tomo_cube {
    int32_t nx, ny, nz; /* voxels per axis, each in [1, 2^24], product <= 2^30 */
    int32_t nframes;    /* time frames held by a cube argument (>= 1)           */
    double box_min[3];  /* box lower corner (box units, e.g. R_sun)             */
    double box_max[3];  /* box upper corner, > box_min on every axis            */
} tomo_cube;

typedef struct tomo_view {
    double obs[3];      /* observer position in the cube frame                  */
    double w[3];        /* unit vector of the tangent point (crpix)             */
    double u[3];        /* unit vector along +column in the tangent plane       */
    double v[3];        /* unit vector along +row in the tangent plane          */
    double cdelt[2];    /* tangent-plane radians per pixel (column, row), != 0  */
    double crpix[2];    /* 0-based pixel position of the tangent point          */
    int32_t ncol, nrow; /* image size, each in 1..65535                         */
    int32_t frame;      /* time frame seen by this view, 0..nframes-1           */
    int32_t reserved;   /* set to 0                                             */
} tomo_view;

/*
 * An opaque sphere, the photosphere of the projector's obstacle variant
 * (Sec. "Fast Parallelized Projector"; integration stops at the photosphere,
 * Sec. "Performance"): every line of sight ends where it enters the sphere's
 * interior.  An observer on or inside the sphere sees nothing; a line that
 * never enters the interior (a tangent line included) is not cut.
 */
typedef struct tomo_obstacle {
    double center[3];  /* cube frame, box units (the Sun's centre: 0, 0, 0)    */
    double radius;     /* > 0 (the photosphere: 1 R_sun)                       */
} tomo_obstacle;

typedef struct tomo_geometry {
    tomo_cube cube;
    int32_t nviews;           /* >= 1                                          */
    int32_t reserved;         /* set to 0                                      */
    const tomo_view *views;   /* HOST array [nviews]                           */
    const uint8_t *data_mask; /* DEVICE [total pixels] or NULL (keep all)      */
    const uint8_t *map_mask;  /* DEVICE [nz][ny][nx] or NULL (keep all); the
                                 same mask applies to every frame               */
    const tomo_obstacle *obstacle; /* HOST pointer or NULL (no obstacle); read
                                      at every call, applies to P, P^T and the
                                      crossing count alike                   */
    const double *gains;      /* HOST [nviews] or NULL (all 1): the gain of the
                                 instrument that took each view, finite
                                 (Eq. two_spacecraft, Eq. lin2space: the rows
                                 of view v are g_v P_v).  Applies to P and P^T
                                 (and so to the solvers and the Thomson
                                 operators), not to the crossing count or the
                                 ray trace, which are geometric            */
} tomo_geometry;

/* Back-projection strategies. */
enum {
    TOMO_BP_AUTO = 0,   /* the tuned default for this geometry                  */
    TOMO_BP_ATOMIC = 1, /* one FP32 atomic add per ray/voxel segment            */
    TOMO_BP_BINNED = 2, /* per-bundle LDS bins, one atomic per voxel per chunk  */
    TOMO_BP_BLOCKED = 3 /* each workgroup owns a voxel block and walks every
                           ray crossing it: LDS bins, one plain store per
                           voxel, no global atomics, deterministic           */
};

/*
 * Projection y = P M x (Eq. lo, Eq. srt).
 *   cube_d:   DEVICE float [nframes][nz][ny][nx]
 *   images_d: DEVICE float [total pixels]; every pixel is written (masked and
 *             missing rays get 0).
 * With a map mask, M x is first written to stream-ordered scratch
 * (hipMallocAsync, the cube's size) and projected by the unmasked walk; if
 * that allocation fails the walk applies the mask itself (same result).
 */
int tomo_project(const tomo_geometry *g, const float *cube_d, float *images_d,
                 tomo_stream stream);

/*
 * Transpose x = M P^T y (or x += M P^T y when accumulate != 0).
 *   images_d: DEVICE float [total pixels]
 *   cube_d:   DEVICE float [nframes][nz][ny][nx]; overwritten unless
 *             accumulate.  TOMO_BP_ATOMIC and TOMO_BP_BINNED add with FP32
 *             atomics, so the last bits may change from run to run;
 *             TOMO_BP_BLOCKED gives the same bits every run.  Non-finite
 *             image values give unspecified (possibly non-finite) results
 *             in the voxels their rays cross.
 *   strategy: TOMO_BP_* (tomo_backproject uses TOMO_BP_AUTO).  The blocked
 *             strategy takes stream-ordered scratch (hipMallocAsync) of
 *             4 * nviews * 64 bytes plus, when blocks are shared between
 *             owners, owners * 4 * nframes * nvox bytes.
 */
int tomo_backproject(const tomo_geometry *g, const float *images_d,
                     float *cube_d, int accumulate, tomo_stream stream);
int tomo_backproject_ex(const tomo_geometry *g, const float *images_d,
                        float *cube_d, int accumulate, int strategy,
                        tomo_stream stream);

/*
 * For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * transpose as tomo_backproject_ex(..., TOMO_BP_BLOCKED, ...), bit for bit,
 * with no allocation of any kind.  Its scratch (4 * nviews * 64 bytes of
 * per-view maxima; owners * 4 * nframes * nvox bytes of partial sums when
 * blocks have several owners; 4 bytes per image pixel of kept-pixel row
 * tables when a data mask is given and footprints are cut to row
 * intervals) lives in one static device array of
 * TOMO_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends.
 *   - The geometry's device tables must already exist: make any other call
 *     with the same geometry first (tomo_count_crossings, tomo_backproject,
 *     ...), as before a stream capture; otherwise TOMO_EINVAL.
 *   - TOMO_EINVAL if the scratch this geometry needs under its tuning
 *     exceeds TOMO_NOALLOC_SCRATCH_BYTES; nothing is launched then.
 *   - Every call on one GPU shares that GPU's array, and each call writes
 *     all the scratch it reads, so nothing carries over between calls; but
 *     calls that overlap in time on one GPU (other streams or threads) race
 *     on it and must be serialised by the caller.
 */
#define TOMO_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int tomo_backproject_noalloc(const tomo_geometry *g, const float *images_d,
                             float *cube_d, int accumulate,
                             tomo_stream stream);

/*
 * Number of positive-length ray/voxel segments walked by one projection
 * (masked pixels excluded): the "voxel crossings" P and P^T each process.
 * Synchronises the stream; *total_h is host memory.
 */
int tomo_count_crossings(const tomo_geometry *g, int64_t *total_h,
                         tomo_stream stream);

/*
 * Test export: the segments the GPU walk produces for one pixel, in order
 * along the ray: flat voxel index (of the view's frame), length, and the
 * parametric length (difference of the ray parameter t at the segment's
 * ends; length = parametric length * |d|).  Runs the same device code as
 * tomo_project on a one-lane launch and synchronises.
 *   idx_h, len_h: HOST arrays of capacity cap; dpar_h: HOST array of
 *   capacity cap or NULL; *n_out = segments written.
 *   Returns TOMO_EINVAL if the pixel is out of range or cap is too small.
 */
int tomo_trace_ray(const tomo_geometry *g, int32_t view, int32_t col,
                   int32_t row, int32_t *idx_h, double *len_h, double *dpar_h,
                   int32_t cap, int32_t *n_out);

/*
 * Launch tuning, process-wide (read by every later launch).  The defaults
 * suit MI355X; tomo_autotune() (or a caller) may change them.
 *   p_bundle, bp_bundle: shape of the pixel bundle one 64-lane wavefront
 *     walks inside a 16x16 workgroup tile: 2 = 4x16, 3 = 8x8, 4 = 16x4 pixels,
 *     0 = the 64 lanes interleaved at a 2-pixel pitch over the whole tile
 *     (p_bundle: P; bp_bundle: the binned and atomic back-projections; the
 *     blocked one walks each footprint 256 pixels at a time in row-major
 *     order and takes no bundle shape).
 *   p_xcd_remap, bp_xcd_remap: order of the tiles (of the voxel-block items
 *     for the blocked back-projection) over the 8 XCDs: 0 = launch order,
 *     1 = one contiguous run per XCD, 2 = runs of 64 per XCD with all XCDs
 *     advancing through the list together (a multi-frame cube then keeps one
 *     frame in the caches at a time).
 *   bp_lds_bins: 64-bit LDS bins per workgroup of the binned
 *     back-projection (512..8192, i.e. 4..64 KiB; larger boxes mean fewer
 *     flushes but fewer resident workgroups).
 *   bp_default: strategy used for TOMO_BP_AUTO (TOMO_BP_BLOCKED,
 *     TOMO_BP_BINNED or TOMO_BP_ATOMIC).
 *   bp_block: voxel block (x, y, z) a workgroup of the blocked
 *     back-projection owns (each 1..256, at most 16384 voxels, one 64-bit
 *     LDS bin each; see bp_threads for what the launch checks).
 *   bp_splits: owners per block in the blocked back-projection, the block's
 *     views dealt round-robin (1..64; 0 = chosen from the block count so
 *     that the launch has about 2048 x 256 / bp_threads workgroups, at most
 *     8 owners).
 *   bp_threads: workgroup size of the blocked back-projection (256, 512 or
 *     1024 lanes).  Larger workgroups own larger blocks for the same
 *     occupancy, so each ray is set up for fewer blocks.  The block's bins
 *     (8 bytes per voxel) must fit the workgroup's LDS with the staging of
 *     its views, or the launch returns TOMO_EINVAL.
 *   p_layout: cube layout P gathers from: 0 = the caller's x-fastest array;
 *     k = 2, 3 or 4 = a bricked copy of it, cubes of 2^k voxels a side (the
 *     bricks in x-fastest order, x fastest inside each), made in
 *     stream-ordered scratch at every call.  The copy costs one pass over
 *     the cube; it pays where the cube is far larger than the caches and
 *     the rays are sparser than the voxels, so that a ray's consecutive
 *     gathers would otherwise each fetch a cache line of their own.
 *   bp_ray_table: 1 = where one geometry serves several blocked
 *     back-projections (tomo_cg_solve, a batch), its rays are set up once
 *     into a table (96 bytes per pixel: in the solve's scratch or workspace,
 *     or held by the batch) that every launch reads, instead of once per
 *     (ray, block) pair; 0 = no table.  Results are the same bit for bit.
 *     Cubes with a side above 2^20 voxels take no table.
 * tomo_set_tuning returns TOMO_EINVAL (and changes nothing) for values out
 * of range.  Not synchronised with launches in flight on other threads.
 */
typedef struct tomo_tuning {
    int32_t p_bundle;
    int32_t p_xcd_remap;
    int32_t bp_bundle;
    int32_t bp_xcd_remap;
    int32_t bp_lds_bins;
    int32_t bp_default;
    int32_t bp_block[3];
    int32_t bp_splits;
    int32_t bp_threads;
    int32_t p_layout;
    int32_t bp_ray_table;
} tomo_tuning;

int tomo_get_tuning(tomo_tuning *out);
int tomo_set_tuning(const tomo_tuning *in);

/*
 * Diagnostic export: number of binned back-projection writes that fell
 * outside their workgroup's LDS box since the last call (each one is a lost
 * contribution, so anything but 0 is a library bug).  Synchronises the
 * device and resets the counter; *count_h is host memory.
 */
int tomo_binning_spills(const tomo_geometry *g, int64_t *count_h);

/*
 * White-light Thomson-scattering operators (Sec. "White Light: Thomson
 * Scattering"; Eq. 4C, Eq. thomson_lo, Eq. brightness, Eq. thomson_direct):
 *   pB = scale O P M n_e,        B = scale (P M' - O P M) n_e,
 * with O = diag(rho_k^2) over pixels (rho the impact parameter of the line
 * of sight) and M, M' diagonal over voxels from Billings' coefficients at
 * sin(Omega) = R_sun / r:
 *   m = ((1 - u) C1 + u C2) / r^4,   m' = 2 ((1 - u) C3 + u C4) / r^2,
 * r and rho in solar radii from the Sun's centre; 0 for voxel centres on or
 * inside the photosphere.  C4 = +1/8 [5 + sin^2 - cos^2/sin (5 - sin^2)
 * ln((1 + sin)/cos)] (the sign its small-angle limit requires).  The map
 * mask multiplies M and M'; masked pixels give 0.  B costs two projections.
 * Work memory: stream-ordered scratch (hipMallocAsync) of one cube and, for
 * B, one more cube and one image set (plus the blocked back-projection's).
 */
typedef struct tomo_thomson {
    double u;             /* limb darkening, in [0, 1]                           */
    double scale;         /* the constant pi sigma I0 / 2 (1: unit-free)         */
    double sun_center[3]; /* cube frame, box units                               */
    double sun_radius;    /* > 0, box units (1 when the box is in R_sun)         */
} tomo_thomson;

enum { TOMO_THOMSON_PB = 0, TOMO_THOMSON_B = 1 };

/* images_d = T n_e (T = T_pB or T_B by kind); ne_d, images_d as in
 * tomo_project. */
int tomo_thomson_project(const tomo_geometry *g, const tomo_thomson *t, int32_t kind,
                         const float *ne_d, float *images_d, tomo_stream stream);

/* ne_d = T^T y (or += with accumulate != 0); deterministic (blocked P^T). */
int tomo_thomson_backproject(const tomo_geometry *g, const tomo_thomson *t, int32_t kind,
                             const float *images_d, float *ne_d, int32_t accumulate,
                             tomo_stream stream);

/*
 * Prior term (Sec. "Single Spacecraft Static Tomography"; Eq. stsrt):
 *   out = [out if accumulate] + lambda_r D^T D x + lambda_t D_t^T D_t x
 * with D the forward differences between in-cube neighbours along x, y and
 * z of each frame (D^T D is the 6-neighbour graph Laplacian with free ends)
 * and D_t the forward difference between consecutive frames.
 *   x_d, out_d: DEVICE float [nframes][nz][ny][nx], must not overlap.
 */
int tomo_apply_prior(const tomo_cube *cube, double lambda_r, double lambda_t,
                     const float *x_d, float *out_d, int accumulate,
                     tomo_stream stream);

/*
 * Voxel heights for the height-weighted prior of Eq. srt_inversion
 * (lambda ||D R e||^2, R the diagonal of voxel heights): the height of a
 * voxel is the distance from its centre to `center` (box units; the Sun's
 * centre) plus `offset` (0: distance from the centre; -1 with a 1 R_sun
 * Sun: altitude above the photosphere).  Both finite.
 */
typedef struct tomo_height {
    double center[3];
    double offset;
} tomo_height;

/*
 * Height-weighted prior (Eq. srt_inversion; Eq. stsrt for time):
 *   out = [out if accumulate] + lambda_r R D^T D R x + lambda_t D_t^T D_t x
 * with R = diag(voxel height) applied to every frame; the temporal term is
 * not weighted.  Heights are computed on the fly from the voxel indices in
 * FP32 (no height array is stored).  h == NULL gives tomo_apply_prior.
 *   x_d, out_d: DEVICE float [nframes][nz][ny][nx], must not overlap.
 */
int tomo_apply_height_prior(const tomo_cube *cube, const tomo_height *h,
                            double lambda_r, double lambda_t,
                            const float *x_d, float *out_d, int accumulate,
                            tomo_stream stream);

/* Learned preconditioner network for the conjugate-gradient inversion: the
 * paper names preconditioning as the untried remedy for CG's slow
 * convergence (Sec. "Smooth Temporal Evolution", closing remarks) and notes
 * that a well-conditioned problem converges faster (Sec. "Bayesian View on
 * Linear Inversion").  Here a network approximates the inverse of the normal
 * operator of Eq. criterion on residuals, inside flexible CG
 * (tomo_cg_solve with precond).  It is a 3x3x3 convolution stack, 1 -> 16
 * -> 16 -> 1 channels with ReLU between layers, zero padding 1.  Parameters are a
 * DEVICE float array of TOMO_CONVNET_NPARAMS values, in this order:
 * w1[16][1][27], b1[16], w2[16][16][27], b2[16], w3[1][16][27], b3[1]
 * (w[cout][cin][kz*9 + ky*3 + kx], cross-correlation like torch.conv3d). */
#define TOMO_CONVNET_NPARAMS 7809

/* DEVICE workspace bytes that tomo_convnet_forward / _loss_grad / _backward
 * need for a cube of this size (one frame); 0 if the cube is invalid. */
size_t tomo_convnet_workspace_bytes(const tomo_cube *cube);

/*
 * out = N(x) on one nx*ny*nz volume (x, out: DEVICE float, x fastest).
 * Every layer runs on MFMA with BF16 operands (the input, the weights and
 * the BF16 hidden activations) and FP32 accumulation.
 * ws_d: DEVICE workspace of at least tomo_convnet_workspace_bytes bytes.
 */
int tomo_convnet_forward(const tomo_cube *cube, const float *params_d,
                         const float *x_d, float *out_d, void *ws_d,
                         size_t ws_bytes, tomo_stream stream);

/*
 * Training gradient of loss = mean((N(x) - target)^2) over the volume:
 * grad_d (DEVICE float[TOMO_CONVNET_NPARAMS]) receives d loss / d params
 * (same layout as the parameters); *loss_h (HOST, may be NULL) the loss,
 * which makes the call synchronise the stream.
 */
int tomo_convnet_loss_grad(const tomo_cube *cube, const float *params_d,
                           const float *x_d, const float *target_d,
                           float *grad_d, double *loss_h, void *ws_d,
                           size_t ws_bytes, tomo_stream stream);

/*
 * Parameter gradient for a caller-given output gradient: grad_d receives
 * sum_v dout[v] * d N(x)[v] / d params, i.e. the gradient of any loss whose
 * derivative with respect to the network output is dout_d (DEVICE float, one
 * value per voxel of x).  The preconditioner is trained this way on the
 * energy-norm error 0.5 (N(r) - e)^T A (N(r) - e), for which dout = A (N(r) - e)
 * comes from tomo_project, tomo_backproject and tomo_apply_prior.  Same
 * activations and precision as tomo_convnet_loss_grad; does not synchronise.
 */
int tomo_convnet_backward(const tomo_cube *cube, const float *params_d,
                          const float *x_d, const float *dout_d, float *grad_d,
                          void *ws_d, size_t ws_bytes, tomo_stream stream);

/* One Adam update (Kingma & Ba) of n parameters in place; step counts from
 * 1; m_d, v_d are the DEVICE moment buffers (zero before the first step). */
int tomo_adam_step(float *params_d, const float *grad_d, float *m_d, float *v_d,
                   int32_t n, int32_t step, double lr, double beta1,
                   double beta2, double eps, tomo_stream stream);

typedef struct tomo_cg_params {
    double lambda_r;       /* spatial prior weight (>= 0)                        */
    double lambda_t;       /* temporal prior weight (>= 0; needs nframes > 1)    */
    int32_t max_iter;      /* iteration limit (>= 0)                             */
    int32_t x0_given;      /* 1: x_d holds the starting point; 0: start at 0     */
    double rtol;           /* stop when ||b - A x|| <= rtol ||b|| (0: never)      */
    int32_t check_every;   /* host convergence check period (iterations, >= 1);
                              with rtol > 0, tomo_cg_solve shortens an interval
                              to the iterations the residual's decay over the
                              last interval predicts are left                 */
    int32_t use_graph;     /* 1: replay each check interval from a HIP graph     */
    const float *precond;  /* DEVICE convnet parameters, or NULL for plain CG    */
    int32_t fallback_window; /* FCG: restart as plain CG after this many
                                iterations without a residual decrease (>= 1)   */
    int32_t bp_strategy;   /* TOMO_BP_*                                          */
    double min_drop;       /* FCG: a residual "decreases" if it falls below
                              (1 - min_drop) times the previous one              */
    float *record_x;       /* DEVICE [record_count][voxels] or NULL: iterate x_k,
                              k = 0..record_count-1 (training data)              */
    float *record_r;       /* DEVICE [record_count][voxels] or NULL: residual r_k */
    int32_t record_count;  /* iterates to record (>= 0)                          */
    int32_t reserved;
    const tomo_height *height; /* HOST pointer or NULL: spatial prior
                                  lambda_r R D^T D R (Eq. srt_inversion)
                                  instead of lambda_r D^T D                  */
    void *workspace;       /* DEVICE, 256-byte aligned, or NULL: memory for all
                              of the solve's device buffers (see
                              tomo_cg_workspace_bytes); NULL takes stream-
                              ordered scratch (hipMallocAsync) per call      */
    size_t workspace_bytes; /* size of workspace                              */
} tomo_cg_params;

typedef struct tomo_cg_report {
    int32_t iters;         /* iterations performed                               */
    int32_t status;        /* TOMO_OK, TOMO_ENOCONV or TOMO_ENONFINITE           */
    int32_t fell_back;     /* FCG: iteration of the switch to plain CG, or -1    */
    int32_t n_project;     /* projections applied (for throughput accounting)    */
    int32_t n_backproject; /* back-projections applied                           */
    int32_t reserved;
    double rel_res;        /* recursive ||r_k|| / ||b|| at exit                  */
    double true_rel_res;   /* ||b - A x|| / ||b|| recomputed at exit             */
    double bnorm;          /* ||b||                                              */
    double ms_project;     /* total time of projection kernels (HIP events)      */
    double ms_backproject; /* total time of back-projection kernels              */
    double *history;       /* HOST [history_cap] or NULL: ||r_k||/||b||, k = 0.. */
    int32_t history_cap;
    int32_t history_len;   /* entries written                                    */
    int32_t time_kernels;  /* input: 1 to time P and P^T launches with events    */
    int32_t reserved2;
} tomo_cg_report;

/*
 * Conjugate-gradient solution of the normal equations of Eq. criterion /
 * Eq. stsrt,  A x = b  with  A = M (P^T G^2 P + lambda_r R D^T D R +
 * lambda_t D_t^T D_t) M  and  b = M P^T G y  (the map mask M restricts the
 * unknowns; G holds the geometry's gains, Eq. srt_multiple_inv; R = I
 * unless params->height is set, Eq. srt_inversion).
 * Textbook CG (FP32 vectors, FP64 dot products and scalars, kept on the
 * device).  Non-finite values in y (unmasked pixels) are reported as
 * status TOMO_ENONFINITE without iterating.  With a preconditioner network,
 * flexible CG with z = ||r|| N(r/||r||)
 * and the Polak-Ribiere beta, falling back to plain CG after
 * fallback_window non-decreasing iterations or when z.r <= 0.
 *   y_d: DEVICE float [total pixels]
 *   x_d: DEVICE float [nframes][nz][ny][nx]: start point if x0_given, and
 *        the solution on return (masked voxels are 0).
 * use_graph = 1 runs the solve as a batch of one (tomo_batch_cg_solve:
 * graph-captured iterations, blocked P^T); it cannot be combined with a
 * preconditioner or recording (TOMO_EUNSUPPORTED).
 * Synchronises the stream.  Returns TOMO_OK when the call ran (the report's
 * status says whether it converged), or an error before/while running.
 */
int tomo_cg_solve(const tomo_geometry *g, const float *y_d, float *x_d,
                  const tomo_cg_params *p, tomo_cg_report *rep,
                  tomo_stream stream);

/* Default parameters: lambda_r 1e-2, max_iter 50, check_every 10,
 * fallback_window 3, min_drop 1e-6, everything else 0 / NULL. */
void tomo_cg_default_params(tomo_cg_params *p);

/*
 * Bytes of device workspace tomo_cg_solve(g, ..., p, ...) takes when
 * p->workspace is set (the vectors of Eq. criterion's CG, the reductions'
 * partials, the blocked P^T's scratch and, if the tuning's bp_ray_table is
 * set, its ray table, P's bricked copy of the iterate if the geometry's
 * tuning walks bricks, and the network's activations with a
 * preconditioner).  The figure depends on the launch tuning in effect for
 * g's size class: query again after tomo_autotune or tomo_set_tuning.
 * Returns 0 for invalid arguments and for use_graph = 1 (a batch of one
 * takes its own memory; tomo_cg_solve refuses a workspace with it).  With a
 * workspace the solve allocates no device memory (the first call on a new
 * geometry still uploads its view table, as every call does); a workspace
 * smaller than this figure is rejected with TOMO_EINVAL.
 */
size_t tomo_cg_workspace_bytes(const tomo_geometry *g, const tomo_cg_params *p);

/*
 * Autotuner (the batched launches of Eq. srt_t and every single-system call
 * take their launch shapes from it).  Times on this geometry the P
 * candidates (wavefront bundles, XCD remap on/off, cube layouts) and the
 * P^T candidates (blocked over block shapes for 256-, 512- and 1024-lane
 * workgroups, owner counts and the XCD remap; binned; atomic), each over
 * `reps` launches through the same paths tomo_project and tomo_backproject
 * take, on a cube of ones and its own projection (tomo_autotune) or on the
 * caller's cube and images (tomo_autotune_data).  The fastest P and P^T
 * candidates are then timed against the process-wide tuning in alternation
 * and kept only if at least 1% faster there; the result becomes the tuning
 * of the geometry's size class (the cube's largest side, the pixels per
 * view and the view count, each rounded up to a power of two, and whether
 * the cube has frames), used by later launches on any geometry of that
 * class instead of the process-wide tuning.
 *   reps: 1..100.  out: HOST, may be NULL.  cube_d, images_d: DEVICE, laid
 *   out as for tomo_project / tomo_backproject, read only.  Synchronises the
 *   stream; takes stream-ordered scratch of about two cubes, two image sets
 *   and the largest owner partials.
 */
int tomo_autotune(const tomo_geometry *g, int32_t reps, tomo_tuning *out,
                  tomo_stream stream);
int tomo_autotune_data(const tomo_geometry *g, const float *cube_d,
                       const float *images_d, int32_t reps, tomo_tuning *out,
                       tomo_stream stream);
/* Tuning in effect for g (*tuned = 1 if it comes from the autotuner). */
int tomo_get_class_tuning(const tomo_geometry *g, tomo_tuning *out,
                          int32_t *tuned);
/* Forget every autotuned size class. */
void tomo_autotune_clear(void);

/*
 * Batched persistent launches over independent systems: the time-frame
 * cubes of one time-dependent reconstruction, whose projector is
 * block-diagonal over the frames (Eq. srt_t, coupled only through the
 * temporal prior of Eq. stsrt), plus independent reconstructions of other
 * sizes.  One persistent P^T kernel (owner-computes, as TOMO_BP_BLOCKED)
 * drains device work queues of (system, frame, voxel block, owner) items
 * covering every system; P runs each system's own launch (the projection
 * needs no queue).  Each system uses the launch shape of its size class
 * (tomo_autotune) as it was when the batch was created, and its results
 * equal the per-system calls with that tuning (tomo_project;
 * tomo_backproject_ex with TOMO_BP_BLOCKED) bit for bit.
 *   systems: HOST array of nsystems geometries (1..32); their masks (DEVICE)
 *   must stay valid while the batch exists, their view arrays need not.
 * The batch owns its device work queues and scratch, and the ray tables of
 * the systems whose tuning sets bp_ray_table (96 bytes per pixel, built
 * when the batch is created, which then synchronises the device): use it
 * from one stream at a time.  tomo_batch_destroy synchronises the device.
 */
typedef struct tomo_batch_s *tomo_batch;
int tomo_batch_create(const tomo_geometry *systems, int32_t nsystems,
                      tomo_batch *out);
void tomo_batch_destroy(tomo_batch b);
/* images_d[k] = P M cubes_d[k] for every system k (HOST arrays of DEVICE
 * pointers, laid out as for tomo_project). */
int tomo_batch_project(tomo_batch b, const float *const *cubes_d,
                       float *const *images_d, tomo_stream stream);
/* cubes_d[k] (+)= M P^T images_d[k] for every system k. */
int tomo_batch_backproject(tomo_batch b, const float *const *images_d,
                           float *const *cubes_d, int accumulate,
                           tomo_stream stream);
/* Writes outside a voxel block's LDS box since the last call (must be 0);
 * synchronises the device and resets the counter. */
int tomo_batch_binning_spills(tomo_batch b, int64_t *count_h);
/* Launch sizes: which 0 = P tiles, 1 = P^T items, 2 = P workgroups (one
 * per tile, over the systems' launches), 3 = P^T workgroups (resident,
 * persistent); -1 for a NULL batch. */
int64_t tomo_batch_items(tomo_batch b, int32_t which);
/*
 * CG on every system at once (plain CG as tomo_cg_solve; each system has
 * its own parameters, state, convergence test, true-residual confirmation
 * and report).  One iteration is the systems' P launches, one batched P^T
 * and three vector kernels per system; converged systems are skipped on
 * the device.
 * check_every and use_graph come from params[0]: with use_graph = 1 the
 * check_every iterations between host checks are captured once as a HIP
 * graph and replayed.  precond and record_* must be unset
 * (TOMO_EUNSUPPORTED); bp_strategy is ignored (always blocked).
 * With reports[0].time_kernels = 1, every report's ms_project and
 * ms_backproject receive the total time of the P launches and of the
 * batched P^T launches of the iterations (shared by all systems;
 * HIP events on the launch stream, recorded as event-record nodes of the
 * graph under use_graph; NaN if the graph could not hold them).
 *   y_d, x_d: HOST arrays of DEVICE pointers.  params, reports: HOST arrays
 *   of nsystems.  Synchronises the stream.
 */
int tomo_batch_cg_solve(tomo_batch b, const float *const *y_d,
                        float *const *x_d, const tomo_cg_params *params,
                        tomo_cg_report *reports, tomo_stream stream);

/*
 * View from helioprojective TAN WCS keywords (the paper's instrument
 * interface, Sec. "Instrument Independence"): observer at distance dsun
 * (box units) and heliographic longitude / latitude (degrees); reference
 * pixel pointing (crval1, crval2) arcsec west / north of Sun centre; image
 * rotation crota (degrees); cdelt in arcsec per pixel; crpix 1-based (FITS).
 * Cube frame: x toward longitude 0 latitude 0, z toward solar north.
 * out is HOST memory; frame is set to 0.
 */
int tomo_view_from_wcs(double dsun, double hgln_deg, double hglt_deg,
                       double crval1_as, double crval2_as, double crota_deg,
                       double cdelt1_as, double cdelt2_as, double crpix1,
                       double crpix2, int32_t ncol, int32_t nrow,
                       tomo_view *out);

/* Validate a geometry without touching the GPU. */
int tomo_validate_geometry(const tomo_geometry *g);

/* Total pixel count of a geometry (0 if invalid). */
int64_t tomo_geometry_pixels(const tomo_geometry *g);

/* Free the cached device view tables. */
void tomo_release_cache(void);

const char *tomo_status_string(int status);
const char *tomo_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TOMO_H */
