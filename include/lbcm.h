/*
 * lbcm — MI355X (gfx950) library for the hybrid central-moments / BGK lattice Boltzmann scheme
 * for the coupled Cahn-Hilliard--Navier-Stokes equations of De Rosis, Saito, Kaneko and Abe,
 * "Central-moments-based lattice Boltzmann scheme for coupled Cahn-Hilliard--Navier-Stokes
 * equations" (arXiv:1803.11345).
 *
 * One handle owns one D2Q9 lattice of nx * ny nodes carrying two population sets: f (flow,
 * collided in the non-orthogonal central-moment basis of Eq. (15) with relaxation Eq. (17))
 * and g (order parameter, BGK relaxation Eq. (7) to the equilibrium of Eqs. (9)-(10)).
 * One call of lbcm_step advances the whole lattice by one time step (Eqs. (4)-(5)).
 *
 * Conventions shared by every entry point
 *   - Planes are row-major [ny][nx], x fastest, node (x, y) at index y * nx + x.
 *   - Directions i = 0..8 follow the paper: c_x = {0,1,0,-1,0,1,-1,-1,1},
 *     c_y = {0,0,1,0,-1,1,1,-1,-1}.
 *   - Every call returns an int status (LBCM_OK or a negative LBCM_E* code); no exception
 *     crosses the boundary.  After an error lbcm_last_error(h) returns a message.
 *   - A handle is not thread-safe; separate handles are independent.  Work is queued on the
 *     handle's HIP stream (params.stream, NULL = the null stream) and runs asynchronously
 *     unless a call says it synchronises.
 *   - Host pointers are only read or written during the call; the caller keeps ownership.
 */
#ifndef LBCM_H
#define LBCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBCM_OK = 0,
    LBCM_EINVAL = -1,    /* bad size, parameter or argument */
    LBCM_ENOMEM = -2,    /* device allocation failed */
    LBCM_EHIP = -3,      /* a HIP runtime call failed */
    LBCM_EDIVERGED = -4, /* a non-finite density or order parameter was detected */
    LBCM_ESTATE = -5     /* call out of order (e.g. step before init) */
};

enum { LBCM_BC_PERIODIC = 0, LBCM_BC_WALLS = 1 };

/* Storage precision of the populations.  FP64 computes in double; the others compute in float. */
enum {
    LBCM_FP64 = 0,
    LBCM_FP32 = 1,         /* f_i - w_i and g_i in float */
    LBCM_FP16_SHIFTED = 2, /* f_i - w_i and g_1..g_8 stored as IEEE half, g_0 as float */
    LBCM_BF16_SHIFTED = 3  /* the same planes stored as bfloat16, g_0 as float */
};

typedef struct lbcm_params {
    int32_t nx, ny;      /* lattice size, >= 1 each */
    int32_t bc_y;        /* LBCM_BC_PERIODIC, or LBCM_BC_WALLS: half-way bounce-back walls at
                            y = -1/2 and y = ny - 1/2 for both f and g (moving along x at the
                            wall velocities below), phi in the ghost rows from the wall
                            gradient; x is always periodic */
    int32_t precision;   /* LBCM_FP64 or LBCM_FP32 (others: see the enum) */
    double a, gamma;     /* free-energy constants: mu = a(-phi + phi^3) - gamma Lap(phi) */
    double mobility;     /* M = (1/omega_phi - 1/2) Gamma c_s^2 */
    double Gamma;        /* Gamma of the g equilibrium, Eq. (9) */
    double nu_l, nu_g;   /* kinematic viscosities at phi = +1 and phi = -1 */
    double omega3;       /* relaxation rate of k3 (bulk viscosity), in (0, 2); 1 recommended */
    double force_x, force_y; /* uniform body force (Guo half-step; 0 = the paper's scheme) */
    double wall_vx_bottom;   /* x velocity of the wall at y = -1/2 (bc_y = LBCM_BC_WALLS; shear test) */
    double wall_vx_top;      /* x velocity of the wall at y = ny - 1/2 */
    double wall_gradient;    /* d_perp phi_w of the contact-angle test at both walls, along the
                                normal into the fluid: the ghost row behind a wall holds the first
                                (last) row's phi minus this value (0: zero normal gradient) */
    int32_t k8_variant;  /* 0: k8 equilibrium from its definition (-gamma |grad phi|^2 / 6);
                            1: the printed -gamma Lap(phi) / 6 of Eq. (16) */
    int32_t check_every; /* > 0: lbcm_step synchronises every check_every steps and at its end
                            and returns LBCM_EDIVERGED once a non-finite rho or phi was seen;
                            0: no check (lbcm_diag still reports it) */
    int32_t tile_rows;   /* step-kernel tile height in wave rows, 0 = default; a wave row covers
                            one lattice row, or two with 16-bit storage on lattices of 2^22
                            nodes or more (lbcm_tile_rows_per_wave) */
    int32_t tile_wx;     /* step-kernel tile width in waves of 64 columns, 0 = default;
                            tile_wx * tile_rows is capped at 16 (FP32, 16-bit) or 8 (FP64) waves.
                            Defaults (wx x rows): 8 x 2 on small lattices; from 2^20 nodes
                            (FP32) or 2^22 (the others) FP32 4 x 3, FP64 2 x 4, 16-bit 4 x 3
                            (two-row waves) */
    void *stream;        /* hipStream_t to queue work on; NULL = null stream */
    void *workspace;     /* optional caller-owned device memory of lbcm_workspace_size() bytes,
                            256-byte aligned; NULL = the library allocates and frees it */
    size_t workspace_bytes;
} lbcm_params;

typedef struct lbcm_diagnostics {
    double sum_phi;      /* sum of phi over the lattice (FP64 accumulation) */
    double sum_abs_phi;  /* sum of |phi| */
    double sum_rho;      /* sum of rho */
    double sum_jx;       /* sum of rho v_x with v = (sum f c + F/2) / rho */
    double sum_jy;
    double max_u;        /* max |v| */
    int64_t nonfinite;   /* number of nodes with a non-finite rho or phi */
    int64_t step;        /* steps taken since lbcm_init */
    double max_du;       /* max |v(t) - v(t-1)|: the largest change of the velocity over the last
                            step (the steady-state measure of a driven channel), from the two
                            population copies the handle keeps; NaN when the spare copy does not
                            hold the previous step's state: before the first step after lbcm_init,
                            lbcm_set_state or lbcm_copy_state, and after lbcm_fields,
                            lbcm_populations or a tile timing, which stage through that copy */
} lbcm_diagnostics;

typedef struct lbcm_handle lbcm_handle;

/* Device bytes needed for a lattice with these parameters (0 if the parameters are invalid). */
size_t lbcm_workspace_size(const lbcm_params *p);

/* Validate the parameters, allocate (or adopt) device memory and return a handle in *out.
   Errors: LBCM_EINVAL (nx, ny < 1, a population set (9 planes) of 4 GiB or more, nu <= 0, mobility <= 0, Gamma <= 0,
   omega3 outside (0, 2), unknown bc/precision, workspace too small or misaligned),
   LBCM_ENOMEM, LBCM_EHIP.  On error *out is NULL. */
int lbcm_create(const lbcm_params *p, lbcm_handle **out);

/* Set f = f^eq and g = g^eq of the given macroscopic state (Eqs. (8)-(10) with the gradient and
   Laplacian of phi0 from Eq. (12)): host planes of nx * ny doubles.  rho0, ux0, uy0 may be NULL
   (meaning 1, 0, 0).  Resets the step counter and the divergence flag.  Synchronises. */
int lbcm_init(lbcm_handle *h, const double *phi0, const double *rho0, const double *ux0,
              const double *uy0);

/* As lbcm_init, with the planes in device memory (read on the handle's stream; asynchronous). */
int lbcm_init_device(lbcm_handle *h, const double *phi0, const double *rho0, const double *ux0,
                     const double *uy0);

/* Queue nsteps >= 0 time steps (one fused kernel launch per step).  Asynchronous unless
   check_every > 0.  Errors: LBCM_ESTATE before lbcm_init, LBCM_EINVAL for nsteps < 0,
   LBCM_EDIVERGED (check_every > 0 only). */
int lbcm_step(lbcm_handle *h, int64_t nsteps);

/* Macroscopic fields of the current state into host planes of nx * ny doubles (any pointer may
   be NULL): phi = sum g, rho = sum f, v = (sum f c + F/2) / rho and the bulk pressure p0 of
   Eq. (13).  Synchronises. */
int lbcm_fields(lbcm_handle *h, double *phi, double *rho, double *ux, double *uy, double *p0);

/* As lbcm_fields, into device planes (asynchronous). */
int lbcm_fields_device(lbcm_handle *h, double *phi, double *rho, double *ux, double *uy,
                       double *p0);

/* The post-streaming populations f_i(x, t) and g_i(x, t) of the current state (the state the
   paper's step starts from) as 9 host planes each, FP64, layout [i][y][x]; either pointer may be
   NULL.  Synchronises. */
int lbcm_populations(lbcm_handle *h, double *f, double *g);

/* FP64 reductions of the current state (deterministic order): sums over the nodes of phi, |phi|,
   rho and rho v, the maxima of |v| and of |v(t) - v(t-1)|, with v = (sum f c + F/2) / rho as
   defined after Eq. (14).  Synchronises. */
int lbcm_diag(lbcm_handle *h, lbcm_diagnostics *out);

/* For callers that cannot allocate device memory (code under graph capture, tight serving
   loops, harnesses that forbid hipMalloc): the diagnostics of lbcm_diag for a state held in the
   caller's device memory, without a handle and without any allocation.  f and g are the two
   population sets as lbcm_get_state lays them out (f: 9 planes, g: 9 planes, pull layout, f
   shifted by the weights, storage precision of p->precision), each aligned to its widest element
   (8 bytes for FP64, 4 otherwise); f_prev, optional, is the f set of the step before, for max_du
   (NaN when f_prev is NULL).  Only nx, ny, bc_y, precision, force and the wall parameters of *p
   are used (p must pass lbcm_create's checks); work runs on p->stream, and the call
   synchronises it.  out->step is set to `step`.
   The partial sums live in a fixed device array of 65,600 bytes that the library holds on each
   GPU for the life of the process (any lattice size fits: the kernels stride over the nodes).
   Calls on the same GPU share that array: calls that overlap in time on one GPU (other host
   threads, other streams) race and must be serialised by the caller.  Errors: LBCM_EINVAL (bad
   parameters, NULL or misaligned pointers), LBCM_EHIP; the message is lbcm_last_error(NULL). */
int lbcm_diag_state(const lbcm_params *p, const void *f, const void *g, const void *f_prev, int64_t step,
                    lbcm_diagnostics *out);

/* Streaming reference for the step kernel's roofline (a measurement, not part of the method): one
   launch reads `planes` (9 or 18) planes of n floats from src and writes them to as many planes of
   dst, one element per lane, non-temporal stores: the step's access pattern without its shifted
   pulls, halo reads and arithmetic.  *ms receives the average time of `reps` launches on
   `stream` (after one untimed launch).  src and dst are device buffers of planes * n floats.
   Synchronises.  Errors: LBCM_EINVAL, LBCM_EHIP (message in lbcm_last_error(NULL)). */
int lbcm_stream_probe(const float *src, float *dst, size_t n, int32_t planes, int32_t reps, void *stream, float *ms);

/* Bytes of the raw population state: 18 planes (f_0..f_8 then g_0..g_8) in storage precision. */
/* The raw state is in pull layout (plane i at node x holds the post-collision value of the
   previous step at its origin node x) and f is stored shifted, as f_i - w_i. */
size_t lbcm_state_size(const lbcm_handle *h);

/* Copy the raw populations out of / into the handle (host buffer of lbcm_state_size bytes;
   values as stored: pull layout, f shifted by the weights).  lbcm_set_state also marks the
   handle initialised and sets the step counter to step.  Both synchronise. */
int lbcm_get_state(lbcm_handle *h, void *host, size_t bytes);
int lbcm_set_state(lbcm_handle *h, const void *host, size_t bytes, int64_t step);

/* Free the handle and the memory it allocated (a caller workspace is left alone). */
int lbcm_destroy(lbcm_handle *h);

/* Message of the last error on h (or of the last failed lbcm_create when h is NULL). */
const char *lbcm_last_error(const lbcm_handle *h);

/* Pick the step kernel's tile shape by timing: every (tile_wx, tile_rows) split with tile_wx a
   power of two up to the lattice width and tile_rows a power of two or three times one is run
   `trials` times (reading the current populations and writing the spare copy, so the state does
   not change), and the fastest is kept in the handle.  Needs lbcm_init first.  Synchronises. */
int lbcm_autotune(lbcm_handle *h, int trials);

/* Device-to-device copy of src's populations into dst (same nx, ny and precision; other physics
   may differ); dst's step counter becomes `step` and its divergence flag is cleared.  Queued on
   dst's stream (after synchronising src's stream if they differ).  Errors: LBCM_EINVAL,
   LBCM_ESTATE (src before lbcm_init), LBCM_EHIP. */
int lbcm_copy_state(lbcm_handle *dst, const lbcm_handle *src, int64_t step);

/* Steps taken since lbcm_init (or the step given to lbcm_set_state / lbcm_copy_state); -1 for
   a NULL handle. */
int64_t lbcm_step_count(const lbcm_handle *h);

/* Copy of the parameters the handle was created with into *out (stream: the handle's stream;
   workspace: as given at creation, NULL when the library allocated it). */
int lbcm_info(const lbcm_handle *h, lbcm_params *out);

/* Tile shape the step kernel uses (after clamping to the lattice): waves across, wave rows down. */
int lbcm_tile_shape(const lbcm_handle *h, int32_t *wx, int32_t *rows);

/* Lattice rows each wave of the step kernel updates: 2 with 16-bit storage on lattices of at least
   2^22 nodes (bandwidth-bound; a wave then has as many bytes in flight as an FP32 wave), else 1. */
int lbcm_tile_rows_per_wave(const lbcm_handle *h, int32_t *rpw);

/* ---------------------------------------------------------------------------------------------
   Ensembles: many independent lattices (boxes) of any sizes, boundaries, forces and viscosities,
   advanced together by one launch per time step that covers every tile of every box.  Each box
   is an ordinary handle (lbcm_batch_box) whose memory lives in the batch: initialise it with
   lbcm_init, read it with lbcm_fields / lbcm_diag / lbcm_populations.  All boxes share the
   precision and the stream (a NULL stream gets a stream of the batch, needed for graph capture).
   Not thread-safe; lbcm_step on a box handle advances that box alone (the batch notices). */
typedef struct lbcm_batch lbcm_batch;

/* nboxes parameter sets (workspace fields ignored).  Errors: LBCM_EINVAL (any box invalid,
   mixed precision or stream), LBCM_ENOMEM, LBCM_EHIP. */
int lbcm_batch_create(const lbcm_params *boxes, int32_t nboxes, lbcm_batch **out);

/* Handle of box i (owned by the batch; do not destroy it), NULL if i is out of range. */
lbcm_handle *lbcm_batch_box(lbcm_batch *b, int32_t i);

/* Advance every box by nsteps with one kernel launch per step (every box must be initialised).
   With graphs enabled (the default) pairs of steps are replayed from a captured hipGraph.
   Asynchronous, unless a box has check_every > 0: then the call synchronises every c steps (c
   the shortest positive check_every of the boxes) and at its end, and returns LBCM_EDIVERGED
   once any box has seen a non-finite rho or phi (the message names the first such box; each
   box's flag is cleared by lbcm_init, lbcm_set_state and lbcm_copy_state of that box). */
int lbcm_batch_step(lbcm_batch *b, int64_t nsteps);

/* The same steps as single-box launches, box after box (the baseline the batched launch is
   measured against). */
int lbcm_batch_step_looped(lbcm_batch *b, int64_t nsteps);

/* The same steps as single-box launches, the boxes of each step dealt round-robin to nstreams
   streams (1 .. 64; default priority, created for the call) forked from and joined back to the
   batch's stream after every step, so that the boxes of one step may run concurrently: the
   baseline that separates what one launch per step gains from concurrency and from launch count.
   The result equals lbcm_batch_step's bit for bit.  nstreams = 1 is lbcm_batch_step_looped.
   Synchronises.  Errors: LBCM_EINVAL for nsteps < 0 or nstreams outside [1, 64], LBCM_EHIP,
   and a box's own LBCM_EDIVERGED (check_every > 0) naming the box. */
int lbcm_batch_step_looped_streams(lbcm_batch *b, int64_t nsteps, int32_t nstreams);

/* Autotuner: for each box size, the fastest tile split of a workgroup of 8, 12 or 16 waves (timed
   on that box), then the workgroup size and the tile order (see lbcm_batch_set_order)
   of the batched launch by timing whole launches; the boxes' own tiles (lbcm_step,
   lbcm_batch_step_looped) become the same tiles, or with 16-bit storage, whose single-lattice
   kernel differs from the batched one, the fastest split for that kernel per box size.  Timing
   runs read the current populations and write the spare copies, so no state changes.
   Synchronises. */
int lbcm_batch_autotune(lbcm_batch *b, int32_t trials);

/* Enable (1, default) or disable (0) hipGraph replay in lbcm_batch_step. */
int lbcm_batch_set_graph(lbcm_batch *b, int32_t enable);

/* Launch schedule of lbcm_batch_step: 0 (default) one launch per step (graph replays of step
   pairs); 1 one persistent launch for all the steps of a call, workgroups taking the tiles of all
   boxes from a global counter in step order, with a grid barrier between steps (a cooperative
   launch of the resident number of workgroups); 2 one persistent launch with a dataflow
   schedule: per-tile step counters, a tile starts step s once every tile its reads or writes
   reach has finished step s - 1 (no barrier; the work is handed out in step order, so every wait
   is on a running workgroup).  Waits are bounded: a launch whose wait gives up (never expected)
   makes lbcm_batch_step return LBCM_EHIP with the boxes' state undefined.  The persistent
   schedules synchronise at the end of every launch (one per call, or one per check_every
   steps).  The schedule changes no result.  Errors: LBCM_EINVAL. */
int lbcm_batch_set_persistent(lbcm_batch *b, int32_t mode);

/* Order of the tiles in the batched launch: 0 the boxes in turn, 1 largest boxes first (default),
   2 one XCD per box (boxes dealt largest first to the XCD with the fewest tiles; a box's halo
   lines are then hits in that XCD's L2).  The order changes no result.  Errors: LBCM_EINVAL. */
int lbcm_batch_set_order(lbcm_batch *b, int32_t order);

/* Current launch configuration: waves per workgroup, tile order, number of tiles, and per box
   the tile shape (arrays of nboxes entries; any pointer may be NULL). */
int lbcm_batch_info(const lbcm_batch *b, int32_t *waves, int32_t *order, int32_t *ntiles, int32_t *wx,
                    int32_t *rows);

/* Free the batch, its boxes and its memory. */
int lbcm_batch_destroy(lbcm_batch *b);

/* Message of the last error on b (or of the last failed lbcm_batch_create when b is NULL). */
const char *lbcm_batch_last_error(const lbcm_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* LBCM_H */
