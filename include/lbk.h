/*
 * lbk.h -- C ABI of the MI355X (gfx950) Klinkenberg lattice Boltzmann library.
 *
 * The library advances the generalized lattice Boltzmann model of Chen et
 * al. (arXiv:1411.7051) for gas flow in tight porous media: a D2Q9 BGK
 * stream-and-collide sweep per time step (Eq. 12) with Guo's porous
 * equilibrium and forcing (Eqs. 14-15), moments and explicit velocity
 * (Eqs. 16-17), and the apparent permeability k_a = k f_c(Kn) of Eq. 3 with
 * the second-order Beskok-Karniadakis/Civan factor (Eqs. 6-7) evaluated at
 * a local Knudsen number Kn = kn0 * rho_ref / rho (Eq. 5 with Eq. 10:
 * the mean free path scales as 1/p).  The force is Eq. 8, or Eq. 2 when the
 * Forchheimer function f_eps is non-zero.
 *
 * Conventions
 *  - Lattice units: dx = dt = 1, c = 1, cs^2 = 1/3, nu = (tau - 1/2)/3.
 *  - Field arrays are row-major [ny][nx], x fastest, float32, unpadded.
 *  - k = +inf marks a node with no Darcy drag (free fluid, Sec. III);
 *    eps = 0 marks an impermeable node (infinite drag, zero velocity).
 *  - Walls are half-way bounce-back; a pressure boundary imposes rho_in on
 *    column 0 and rho_out on column nx-1 by non-equilibrium extrapolation
 *    from the neighbouring column (Sec. IV.A: pressure-driven plates).
 *  - Every call is asynchronous on the HIP stream given at create, except
 *    those that return host scalars, which synchronize that stream.
 *  - Every function returns an lbk_status; on error lbk_last_error() holds a
 *    message for the calling thread.  No exception crosses the ABI.
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef LBK_H
#define LBK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lbk_status {
    LBK_OK = 0,
    LBK_ERR_INVALID_ARG = -1, /* bad description, field value or pointer */
    LBK_ERR_DEVICE = -2,      /* HIP runtime error or no gfx950 device */
    LBK_ERR_OOM = -3,         /* workspace too small */
    LBK_ERR_NONFINITE = -4,   /* a NaN or Inf appeared in the state */
    LBK_ERR_UNSUPPORTED = -5  /* combination not implemented */
} lbk_status;

typedef enum lbk_bc {
    LBK_BC_PERIODIC = 0,
    LBK_BC_WALL = 1,    /* half-way bounce-back (no-slip plates, Sec. IV.A) */
    LBK_BC_PRESSURE = 2 /* x only: rho_in at x = 0, rho_out at x = nx-1 */
} lbk_bc;

/* Element type of the nine stored population planes.  The collide
 * arithmetic is FP32 for every storage type. */
typedef enum lbk_storage {
    LBK_F32 = 0,
    LBK_F16 = 1, /* with a power-of-two scale managed by the library */
    LBK_BF16 = 2
} lbk_storage;

/* Slip correction f_c of the apparent permeability k_a = k f_c (Eq. 3). */
typedef enum lbk_correlation {
    LBK_FC_BKC = 0,         /* second-order Beskok-Karniadakis/Civan, Eqs. 6-7,
                               with slip coefficient slip_b (default -1) */
    LBK_FC_KLINKENBERG = 1, /* first-order Klinkenberg, Eqs. 4-5: 1 + 4 Kn */
    LBK_FC_NONE = 2         /* no slip correction: k_a = k */
} lbk_correlation;

/* How lbk_step (and a gradient's recomputing sweeps and reverse steps)
 * advance a lattice: two or three time steps per pass, the intermediate
 * levels kept in registers (bitwise the result of as many single sweeps),
 * or one step per sweep.  A multi-step pass reads and writes the state
 * once per pass; it pays off on lattices large enough to fill the device. */
typedef enum lbk_pass_mode {
    LBK_PASS_AUTO = 0,     /* three-step passes from 2^22 nodes (FP32), 2^23
                              (FP16/BF16); two-step passes from 2^20 (FP32),
                              2^22 (FP16/BF16); single sweeps below */
    LBK_PASS_TWO_STEP = 1, /* two-step passes whatever the size */
    LBK_PASS_SINGLE = 2,   /* single sweeps */
    LBK_PASS_THREE_STEP = 3 /* lbk_step: three-step passes whatever the size (a
                               remainder of n in a two-step pass or a single
                               sweep); gradients record in three-step passes
                               and reverse in two-step passes */
} lbk_pass_mode;

/* Run description (Sec. IV: plates, heterogeneous media, fractured shale). */
typedef struct lbk_desc {
    int32_t nx, ny;      /* lattice size; nx >= 3 with pressure boundaries */
    int32_t bc_x, bc_y;  /* lbk_bc; bc_y may not be LBK_BC_PRESSURE */
    int32_t storage;     /* lbk_storage */
    int32_t kn_local;    /* 1: Kn = kn0 * rho_ref / rho; 0: Kn = kn0 */
    int32_t init;        /* 0: rest at rho0; 1: rest on the linear density
                            ramp rho_in -> rho_out along x */
    int32_t check_every; /* lbk_step checks the state for NaN/Inf (and, for
                            FP16, re-centres the scale) whenever the
                            lattice's time reaches a multiple of this
                            (default 100; 0 = never).  Each check
                            synchronizes the stream and reads the state
                            once (about 1% of a step's traffic at 100).
                            FP16 starts at the scale 2^20, which holds
                            deviations from 2^-34 to 2^-4 at full
                            precision; runs that leave that range need
                            checks to move the scale */
    double tau;          /* BGK relaxation time (Eq. 12), > 1/2 */
    double gx, gy;       /* external acceleration G (Eqs. 2, 8) */
    double f_eps;        /* Forchheimer geometric function (Eq. 2); 0 = Eq. 8 */
    double rho_in, rho_out; /* pressure-boundary densities */
    double rho0;         /* initial density for a start at rest */
    double rho_ref;      /* density at which kn0 is quoted */
    double slip_b;       /* slip coefficient b of Eq. 6, <= 0 (default -1) */
    int32_t correlation; /* lbk_correlation */
    int32_t pass_mode;   /* lbk_pass_mode: one, two or three steps per pass */
    int32_t band;        /* rows per band of the multi-step passes, forward
                            and reverse, 1..1024; 0 (default) = by size and
                            storage: two-step passes 8 rows at FP32, 10 at
                            FP16/BF16, three-step passes 12 and 24, 16 in
                            reverse, halved down to 2 while a pass
                            would have fewer than 8192 waves.  Any band
                            gives the same result bitwise.  A batch ignores
                            it (its passes take the default bands) */
} lbk_desc;

typedef struct lbk_lattice lbk_lattice;

/* Fill *d with defaults: periodic, FP32, tau 0.8, rho 1, no force, local Kn,
 * the second-order correlation with b = -1, state checks every 100 steps. */
lbk_status lbk_desc_default(lbk_desc *d);

/* Bytes of device workspace lbk_create needs for this description.
 * Size limits (LBK_ERR_UNSUPPORTED beyond them): at most 2^30 nodes with x
 * padded to a multiple of 64, and rows of at most 107,374,144 nodes (the
 * kernels address a row block with 32-bit offsets). */
lbk_status lbk_workspace_size(const lbk_desc *d, size_t *bytes);

/* Create a lattice.  eps, k, kn0: [ny][nx] float32 arrays in host or device
 * memory (kn0 may be NULL, meaning 0); they are copied and validated
 * (0 <= eps <= 1, k > 0 or +inf, kn0 >= 0 and finite) before the call
 * returns.  workspace: caller-owned device memory of ws_bytes >=
 * lbk_workspace_size(), 256-byte aligned, which must outlive the handle.
 * stream: a hipStream_t (NULL = the null stream).  On failure *out is NULL
 * and nothing is left allocated.  The state starts at rest (init). */
lbk_status lbk_create(const lbk_desc *d, const float *eps, const float *k,
                      const float *kn0, void *workspace, size_t ws_bytes,
                      void *stream, lbk_lattice **out);

/* Release the handle (not the workspace).  NULL is accepted. */
lbk_status lbk_destroy(lbk_lattice *lat);

/* Advance n >= 0 time steps of Eq. 12: one fused sweep launch per step,
 * or per two steps in two-step passes (lbk_steps_per_launch), an odd count
 * ending in one single sweep. */
lbk_status lbk_step(lbk_lattice *lat, int64_t n);

/* Number of steps taken since create (or since the loaded state). */
lbk_status lbk_time(const lbk_lattice *lat, int64_t *t);

/* Steps each launch of lbk_step advances, 1, 2 or 3, as the descriptor's
 * pass_mode and the lattice's size and storage decide (a gradient's
 * recording passes follow the same choice, its reverse steps take two where
 * lbk_step takes three). */
lbk_status lbk_steps_per_launch(const lbk_lattice *lat, int32_t *steps);

/* Macroscopic read-out at the current time (Eqs. 16-17 on the post-stream
 * populations, after the boundary override): density and velocity as
 * [ny][nx] float32 into device buffers; any pointer may be NULL. */
lbk_status lbk_read_macroscopic(lbk_lattice *lat, float *rho, float *ux,
                                float *uy);

/* The current post-collision populations f*_i, reconstructed in FP64 as
 * [9][ny][nx] into a device buffer (direction order of Eq. 13). */
lbk_status lbk_read_populations(lbk_lattice *lat, double *f);

/* Global (apparent) permeability of the whole domain by Darcy's law
 * (Sec. IV.A): nu <u_x> / G_x for a body-force drive;
 * eps_b nu (nx-1) <rho u_x> / (cs^2 (rho_in - rho_out)) for a pressure
 * drive, eps_b being the mean porosity of the two pressure columns.
 * Means over every node, accumulated in FP64.  LBK_ERR_INVALID_ARG
 * without a drive to normalise by (rho_in == rho_out, or gx == 0 without
 * pressure columns).  Synchronizes the stream. */
lbk_status lbk_apparent_permeability(lbk_lattice *lat, double *k_app);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the value of
 * lbk_apparent_permeability, within FP64 rounding of the sums (the
 * read-out walks the lattice with a fixed grid of at most 2048 workgroups,
 * so the partial sums are grouped differently).  It calls no hipMalloc,
 * hipFree or other allocating routine and uses neither the lattice's
 * workspace nor its pinned host buffer: its partial sums live in a fixed
 * device array of 12,294 doubles (98 KB) that the library holds on each
 * GPU it runs on until the process ends, and the result is copied straight
 * into *k_app.  Every lattice size fits that array; a layout that did not
 * would be refused with LBK_ERR_UNSUPPORTED.  All calls on one GPU share
 * the array: calls that overlap in time on one GPU (other host threads,
 * lattices on other streams) race and must be serialized by the caller.
 * Makes the lattice's device current for the call.  LBK_ERR_INVALID_ARG
 * without a drive.  Synchronizes the stream. */
lbk_status lbk_apparent_permeability_noalloc(lbk_lattice *lat, double *k_app);

/* FP64 diagnostics: total mass sum f*, x mass flux sum rho u_x, and the
 * residual ||u - u_prev|| / ||u|| against the velocity of the previous
 * lbk_diagnostics call on this handle (+inf on the first call; 0 when the
 * velocity is zero now and was zero then, +inf when it fell to zero).  Any
 * pointer may be NULL.  Synchronizes the stream. */
lbk_status lbk_diagnostics(lbk_lattice *lat, double *mass, double *flux_x,
                           double *residual);

/* Size of a saved state; save copies the state (and the step count) to
 * host or device memory, load restores it into a handle created with the
 * same description.  Both are asynchronous on the stream. */
lbk_status lbk_state_size(const lbk_lattice *lat, size_t *bytes);
lbk_status lbk_save_state(lbk_lattice *lat, void *dst);
lbk_status lbk_load_state(lbk_lattice *lat, const void *src);

/* ---------------------------------------------------------------------
 * Gradients (reverse mode through the discrete time stepping).
 *
 * J is a scalar read-out of the state after n steps; the gradients are
 * dJ / d ln k(x) and, on request, dJ / d ln kn0(x) for every node, with
 * eps and the starting state held fixed (and kn0, resp. k, held fixed: for
 * a medium whose kn0 follows from k through Eq. 11, kn0 ~ k^-1/2, the
 * total derivative is dJ/d ln k - 1/2 dJ/d ln kn0).  The reverse sweep is
 * the exact transpose of the discrete map (pull, pressure-column override,
 * collide of Eqs. 12, 14, 15, 17, 8, 3, 6-7 with the local Kn), evaluated
 * along the forward trajectory, which is recomputed from checkpoints:
 *   - lbk_adjoint_forward runs the n steps (advancing the lattice exactly
 *     as lbk_step would) and stores the state every ckpt_every steps;
 *   - lbk_adjoint_backward recomputes each checkpoint segment (from inner
 *     checkpoints every hist_len steps when hist_len < ckpt_every), records
 *     the per-step linearisation point (rho, j: 12 B per node and step,
 *     hist_len steps at a time) and runs the reverse steps.
 * With hist_len < ckpt_every the forward pass also keeps the inner
 * checkpoints of the last segments, as many as the workspace holds (at
 * least the last one; each further segment takes ceil(ckpt_every /
 * hist_len) state levels beyond lbk_adjoint_workspace_size); the backward
 * pass rebuilds those of the other segments.
 * Cost of the backward pass per step: one recording sweep and one reverse
 * sweep, plus (two-level) about (1 - hist_len/ckpt_every) of a plain sweep
 * in every segment whose inner checkpoints were not kept;
 * lbk_adjoint_plan picks the plan that rebuilds least within a memory
 * budget.
 * With the Forchheimer term (f_eps > 0) the reverse sweep differentiates
 * the quadratic velocity solve of Eq. 2 as well.
 * --------------------------------------------------------------------- */
typedef enum lbk_objective {
    LBK_OBJ_PERMEABILITY = 0, /* the global permeability of
                                 lbk_apparent_permeability (Sec. IV.A) */
    LBK_OBJ_OUTLET_FLUX = 1   /* sum over column x = nx-1 of rho u_x */
} lbk_objective;

/* Device workspace bytes for a gradient over n_steps with checkpoints every
 * ckpt_every steps and a history of hist_len steps (1 <= hist_len <=
 * ckpt_every; hist_len == ckpt_every is the one-level scheme). */
lbk_status lbk_adjoint_workspace_size(const lbk_lattice *lat, int64_t n_steps,
                                      int64_t ckpt_every, int64_t hist_len, size_t *bytes);

/* The checkpoint plan for a gradient over n_steps with checkpoints every
 * ckpt_every steps that fits in budget_bytes and spends the fewest plain
 * sweeps rebuilding inner checkpoints (among equals, the longest history):
 * *hist_len (at most ckpt_every) and, in *bytes (may be NULL), the
 * workspace to pass to lbk_adjoint_forward, which includes the kept inner
 * checkpoints of as many segments as fit.  LBK_ERR_OOM if none fits.
 * Host-only, no device work. */
lbk_status lbk_adjoint_plan(const lbk_lattice *lat, int64_t n_steps, int64_t ckpt_every,
                            size_t budget_bytes, int64_t *hist_len, size_t *bytes);

/* Run n_steps forward from the current state, storing checkpoints in the
 * caller's device workspace (256-byte aligned, ws_bytes >=
 * lbk_adjoint_workspace_size; a larger workspace keeps inner checkpoints
 * of more segments), and return J (host double; synchronizes).
 * The lattice ends at t + n_steps.  The FP16 scale is held fixed and
 * check_every is not applied during these steps. */
lbk_status lbk_adjoint_forward(lbk_lattice *lat, int objective, int64_t n_steps,
                               int64_t ckpt_every, int64_t hist_len, void *ws, size_t ws_bytes,
                               double *J);

/* Gradients of the J of the last lbk_adjoint_forward on this handle (same
 * workspace, no lbk_step or load in between) into device buffers of
 * [ny][nx] float32: dJ_dlnk (required) and dJ_dlnkn0 (NULL to skip it; it
 * is 0 where kn0 = 0).  Leaves the lattice state untouched. */
lbk_status lbk_adjoint_backward(lbk_lattice *lat, void *ws, size_t ws_bytes, float *dJ_dlnk,
                                float *dJ_dlnkn0);

/* ---------------------------------------------------------------------
 * Ensembles: many independent samples stepped together.
 *
 * A batch groups n lattices of uneven size (independent heterogeneous
 * samples, each with its own fields, tau, drive and Kn scale) so that one
 * kernel launch advances every sample by one step (or two, see
 * lbk_batch_set_pass_mode).  The launch walks a list
 * of tiles -- tile_x consecutive x by `rows` consecutive y of one sample --
 * that covers all samples; either one workgroup per tile or a persistent
 * grid of `grid` workgroups each taking a contiguous run of tiles.  Steps
 * can be recorded into HIP graphs of `graph_steps` launches that are
 * replayed.
 * Each sample's update is the same arithmetic as lbk_step on that lattice,
 * so results are bitwise identical to stepping the lattices one by one, for
 * every launch configuration.
 *
 * The lattices stay owned by the caller (they must outlive the batch) and
 * keep working as handles: read-outs, save/load and lbk_step may be used
 * between batch calls.  All of them must share storage, bc_x, bc_y and
 * the stream they were created on; the batch works on that stream.
 * check_every is not applied by lbk_batch_step: a caller that wants the
 * state checks calls lbk_batch_check at its own interval.
 * --------------------------------------------------------------------- */
typedef struct lbk_batch lbk_batch;

/* Device workspace bytes for a batch over lats[0..n-1] (n >= 1). */
lbk_status lbk_batch_workspace_size(lbk_lattice *const *lats, int32_t n, size_t *bytes);

/* Create a batch over lats[0..n-1] in a caller-owned device workspace
 * (256-byte aligned, ws_bytes >= lbk_batch_workspace_size).  The launch
 * configuration starts at 256 x 1 tiles, one workgroup per tile, no
 * graphs. */
lbk_status lbk_batch_create(lbk_lattice *const *lats, int32_t n, void *workspace,
                            size_t ws_bytes, lbk_batch **out);

/* Release the batch (not the lattices or the workspace); NULL accepted. */
lbk_status lbk_batch_destroy(lbk_batch *b);

/* Advance every sample by n >= 0 steps (each lattice's time grows by n). */
lbk_status lbk_batch_step(lbk_batch *b, int64_t n);

/* Launch configuration: tiles of tile_x in {64, 128, 192, 256} (the
 * workgroup size) by rows in 1..64; grid 0 = one workgroup per tile, else a
 * persistent grid of 1..2^20 workgroups; graph_steps 0 = direct launches,
 * else an even number of steps (2..1024) recorded per graph replay.
 * Changing the tiling synchronizes the stream. */
lbk_status lbk_batch_set_launch(lbk_batch *b, int32_t tile_x, int32_t rows, int32_t grid,
                                int32_t graph_steps);
lbk_status lbk_batch_get_launch(const lbk_batch *b, int32_t *tile_x, int32_t *rows,
                                int32_t *grid, int32_t *graph_steps);

/* Steps per launch, as pass_mode does for a lattice (lbk_pass_mode):
 * LBK_PASS_TWO_STEP: two-step passes, the tile list then holding groups of
 * four 60-column strips by a band of rows of each sample (tile_x, rows and
 * grid apply to single steps only, such as the last of an odd count);
 * LBK_PASS_SINGLE: one step per launch; LBK_PASS_AUTO (the default):
 * two-step passes for batches of 2^22 nodes and more, until
 * lbk_batch_autotune has timed both and keeps the faster.  Either way each
 * sample ends bitwise where single steps take it.  Drops recorded graphs
 * when the choice changes.  Batches have no three-step pass:
 * LBK_PASS_THREE_STEP is rejected (LBK_ERR_INVALID_ARG). */
lbk_status lbk_batch_set_pass_mode(lbk_batch *b, int32_t pass_mode);
/* The pass mode set, and the steps per launch in use (1 or 2); either
 * pointer may be NULL. */
lbk_status lbk_batch_get_pass_mode(const lbk_batch *b, int32_t *pass_mode,
                                   int32_t *steps_per_launch);

/* on != 0: every graph replay ends with the per-sample read-out reductions
 * (the FP64 sums behind lbk_batch_apparent_permeability), so that after
 * steps that end in a replay the permeabilities need only a copy of the
 * sums.  Off by default. */
lbk_status lbk_batch_set_graph_readout(lbk_batch *b, int32_t on);

/* Time every candidate -- tile_x in {64, 128, 256} x rows in {1, 4, 8, 16}
 * x one workgroup per tile or persistent grids of 2, 4 and 8 workgroups
 * per compute unit -- over `reps` >= 1 steps each, and keep the fastest
 * (graph_steps unchanged); with pass_mode LBK_PASS_AUTO also the two-step
 * pass (reps passes), kept when its time per step is lower.
 * The samples' states are left untouched: the timed launches re-read the
 * current time level and overwrite only the other one.  best_us (may be
 * NULL) receives the fastest mean time per step in microseconds.
 * Synchronizes the stream. */
lbk_status lbk_batch_autotune(lbk_batch *b, int32_t reps, double *best_us);

/* Global permeability of every sample (as lbk_apparent_permeability of
 * that lattice, bitwise) into host k_app[n], from one batched read-out;
 * NaN for a sample without a drive.  Synchronizes the stream. */
lbk_status lbk_batch_apparent_permeability(lbk_batch *b, double *k_app);

/* NaN/Inf check of every sample (and FP16 scale re-centring); returns
 * LBK_ERR_NONFINITE naming the first bad sample.  Synchronizes. */
lbk_status lbk_batch_check(lbk_batch *b);

/* Gradients of every sample of a batch (the calls above, for all samples at
 * once: recomputing sweeps and reverse steps walk the batch's tile list with
 * its tiling, one workgroup per tile).  Every sample's J and gradient are
 * bitwise those of lbk_adjoint_forward / lbk_adjoint_backward on that
 * lattice alone with the same n_steps, ckpt_every and hist_len.  The
 * workspace holds a per-sample slice plus a descriptor table; as for one
 * lattice, a workspace beyond lbk_batch_adjoint_workspace_size keeps the
 * inner checkpoints of more trailing segments (the same number for every
 * sample), and lbk_batch_adjoint_plan returns the hist_len and workspace
 * size that rebuild least within a budget.  J: host
 * double[n]; dJ_dlnk, dJ_dlnkn0: host arrays of n device pointers to
 * [ny][nx] float32 planes (dJ_dlnkn0 may be NULL).  The samples must not be
 * stepped, loaded or rescaled between forward and backward. */
lbk_status lbk_batch_adjoint_workspace_size(lbk_batch *b, int64_t n_steps, int64_t ckpt_every,
                                            int64_t hist_len, size_t *bytes);
lbk_status lbk_batch_adjoint_plan(lbk_batch *b, int64_t n_steps, int64_t ckpt_every,
                                  size_t budget_bytes, int64_t *hist_len, size_t *bytes);
lbk_status lbk_batch_adjoint_forward(lbk_batch *b, int objective, int64_t n_steps,
                                     int64_t ckpt_every, int64_t hist_len, void *ws,
                                     size_t ws_bytes, double *J);
lbk_status lbk_batch_adjoint_backward(lbk_batch *b, void *ws, size_t ws_bytes,
                                      float *const *dJ_dlnk, float *const *dJ_dlnkn0);

/* Host-side correction factor f_c(Kn) of a correlation in FP64 (Eq. 3's
 * k_a / k; Eqs. 6-7 with slip coefficient slip_b, Eqs. 4-5, or 1), for
 * n >= 0 Knudsen numbers in host memory (finite, >= 0); f_c(0) = 1.  For
 * front ends that map physical conditions to lattice inputs. */
lbk_status lbk_correction_factor(int32_t correlation, double slip_b, const double *kn,
                                 double *fc, size_t n);

/* ---------------------------------------------------------------------
 * Three dimensions: the same model on a D3Q19 lattice.
 *
 * The sweep of lbk_step with nineteen velocities (rest, six axis links with
 * weight 1/18, twelve face diagonals with weight 1/36; cs^2 = 1/3): pull
 * with wrap or half-way bounce-back on each axis, pressure planes at x = 0
 * and x = nx-1 (non-equilibrium extrapolation from the neighbouring plane),
 * Eqs. 14-17 with three-component vectors, the local Kn and the selected
 * slip correlation.  Fields are [nz][ny][nx] float32 (x fastest).  Storage,
 * ownership, streams and errors follow the D2Q9 calls; gradients and
 * batches are D2Q9 only.
 * --------------------------------------------------------------------- */
typedef struct lbk_desc3 {
    int32_t nx, ny, nz;
    int32_t bc_x, bc_y, bc_z; /* lbk_bc; only bc_x may be LBK_BC_PRESSURE */
    int32_t storage;          /* lbk_storage */
    int32_t kn_local;         /* 1: Kn = kn0 * rho_ref / rho; 0: Kn = kn0 */
    int32_t init;             /* 0: rest at rho0; 1: ramp rho_in -> rho_out in x */
    int32_t check_every;      /* NaN check (and FP16 re-scaling) at multiples of this
                                 time (default 100); 0 = never */
    int32_t correlation;      /* lbk_correlation */
    int32_t reserved;         /* must be 0 */
    double tau;
    double gx, gy, gz;        /* external acceleration G */
    double f_eps;             /* Forchheimer function of Eq. 2; 0 = Eq. 8 */
    double rho_in, rho_out, rho0, rho_ref;
    double slip_b;            /* slip coefficient of Eq. 6, <= 0 (default -1) */
} lbk_desc3;

typedef struct lbk_lattice3 lbk_lattice3;

/* Defaults: periodic, FP32, tau 0.8, rho 1, no force, local Kn, Eqs. 6-7,
 * state checks every 100 steps. */
lbk_status lbk3_desc_default(lbk_desc3 *d);
/* Limits: at most 2^30 nodes (x padded to 64), ny nz <= 2^24, rows of at
 * most 53,687,040 nodes. */
lbk_status lbk3_workspace_size(const lbk_desc3 *d, size_t *bytes);
/* As lbk_create, with fields [nz][ny][nx]. */
lbk_status lbk3_create(const lbk_desc3 *d, const float *eps, const float *k, const float *kn0,
                       void *workspace, size_t ws_bytes, void *stream, lbk_lattice3 **out);
lbk_status lbk3_destroy(lbk_lattice3 *lat);
lbk_status lbk3_step(lbk_lattice3 *lat, int64_t n);
lbk_status lbk3_time(const lbk_lattice3 *lat, int64_t *t);
/* FP16 storage: the exponent e of the power-of-two scale 2^e the stored
 * deviations currently carry (20 at creation, re-centred by the state checks
 * of check_every); 0 for FP32 and BF16. */
lbk_status lbk3_scale_exponent(const lbk_lattice3 *lat, int32_t *e);
/* rho and the three velocity components as [nz][ny][nx] float32 device
 * buffers (any may be NULL). */
lbk_status lbk3_read_macroscopic(lbk_lattice3 *lat, float *rho, float *ux, float *uy,
                                 float *uz);
/* Post-collision populations in FP64, [19][nz][ny][nx], into a device buffer. */
lbk_status lbk3_read_populations(lbk_lattice3 *lat, double *f);
/* Global permeability as lbk_apparent_permeability (means over every node;
 * eps_b over the two pressure planes).  Synchronizes. */
lbk_status lbk3_apparent_permeability(lbk_lattice3 *lat, double *k_app);
/* FP64 total mass and x mass flux (either may be NULL).  Synchronizes. */
lbk_status lbk3_diagnostics(lbk_lattice3 *lat, double *mass, double *flux_x);

/* Message of the last failed call on this thread ("" if none). */
const char *lbk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBK_H */
