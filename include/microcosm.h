/*
 * microcosm.h -- C ABI of the MI355X filament-fluid timestep library
 * (libmicrocosm.so).
 *
 * One step advances elastic filament chains immersed in a periodic 2D viscous
 * fluid, following the Methods section of "Microcosmos: Reimagining
 * Artificial Life for the GPU Era" (arXiv 2607.02954):
 *   S0 actuation: time-dependent rest angle (Experiments, Hand-designed
 *      locomotion: sinusoidal wave along the body);
 *   S1 elastic force from position-based Cosserat constraints, a bending pass
 *      (Eq. 1) then a position pass (Eqs. 2-4), iterated;
 *   S2-S4 steric repulsion: node density deposited on the grid, Gaussian
 *      filtered, its gradient gives repulsion (Methods, Fields);
 *   S5 force spread onto the grid (immersed boundary method, Methods,
 *      Fluid-filament Interaction);
 *   S6 D2Q9 lattice Boltzmann update with two-relaxation-time collision
 *      (Methods, Fields; Fluid-filament Interaction);
 *   S7 grid velocity gathered back to the nodes, which are integrated.
 *
 * Conventions shared by every entry point:
 *  - Lattice units: cell (ix, iy) is centred at (ix, iy); the grid is
 *    periodic; grid arrays are row-major [ny][nx] with x fastest.
 *  - All array pointers are DEVICE pointers owned by the caller; they must
 *    stay valid while a world or batch refers to them.  The library never
 *    allocates device memory: all scratch lives in caller-provided workspace
 *    or pool memory, sized with the *_size queries (sim_step_noalloc uses a
 *    static device array of the library instead).
 *  - `stream` arguments are hipStream_t values passed as void*; all work is
 *    enqueued asynchronously on that stream.  Only sim_sync, sim_batch_sync,
 *    sim_batch_retire and sim_create/sim_batch_admit (which read the CSR
 *    offsets back) synchronise.
 *  - Every call returns a sim_status.  SIM_E_INVALID / SIM_E_WORKSPACE /
 *    SIM_E_FULL are detected on the host before any work is enqueued and
 *    leave all state untouched.  sim_last_error() returns a thread-local
 *    message for the last non-OK status.  Nothing aborts or throws across
 *    this boundary.
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef MICROCOSM_H
#define MICROCOSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sim_status {
  SIM_OK = 0,
  SIM_E_INVALID = 1,   /* bad argument, size or layout                         */
  SIM_E_WORKSPACE = 2, /* workspace / pool / checkpoint buffer too small        */
  SIM_E_HIP = 3,       /* a HIP runtime call failed (message in sim_last_error) */
  SIM_E_UNSTABLE = 4,  /* a world produced NaN or |u| > u_max (Mach guard)      */
  SIM_E_STATE = 5,     /* call not valid in the handle's current state          */
  SIM_E_FULL = 6       /* batch has no free slot                                */
} sim_status;

/* sim_params.flags */
/* Particle -> grid transfer (deposit and force spread).  Default (no flag):
 * nodes are binned by the grid tile (side tile_side) of their home cell; every tile
 * reads the bins of its neighbourhood, sums the contributions that reach it
 * in on-chip memory (integer fixed point: results are bitwise reproducible)
 * and writes each cell once.  The two flags are exclusive. */
enum {
  SIM_SPLAT_SORTED = 1u << 0, /* deterministic: counting sort by home cell, fixed-order
                                 segmented sums; results are bitwise reproducible       */
  SIM_SPLAT_DIRECT = 1u << 1  /* global float atomics into HBM accumulators (reference) */
};

/* Physical and numerical constants of one world (host struct, copied). */
typedef struct sim_params {
  int32_t nx, ny;          /* periodic grid, cells; each >= 8                         */
  float tau;               /* relaxation time, viscosity nu = (tau - 1/2)/3, > 0.5   */
  float trt_magic;         /* TRT magic parameter Lambda (default 1/4), > 0          */
  float k_bend;            /* bending stiffness of Eq. 1, in [0, 1]                  */
  float k_stretch;         /* stretch stiffness of Eq. 3, in [0, 1]                  */
  float k_shear;           /* shear blend of Eq. 3, in [0, 1]                        */
  int32_t pbd_iters;       /* PBD iterations per step, >= 0                          */
  float k_elastic;         /* elastic force F_el = k_elastic (y - x)                 */
  float k_repulse;         /* steric repulsion strength                              */
  float sigma_repulse;     /* Gaussian filter width (cells), > 0                     */
  int32_t repulse_radius;  /* Gaussian filter truncation radius, 1..8                */
  float u_max;             /* Mach guard: |u| above this flags the world unstable    */
  uint32_t flags;          /* SIM_SPLAT_SORTED or SIM_SPLAT_DIRECT, else binned      */
  int32_t tile_side;       /* side of the square grid tiles the transfer and filter
                              kernels work on (and of the node bins): 16, 32 or 64;
                              0 means 32.  A tuning choice: results do not depend
                              on it beyond rounding (binned: not at all).          */
  float energy_rate;       /* energy field (sim_arrays.energy): fraction of the
                              sensed energy a node collects per step, in [0, 1];
                              0 disables the field                                 */
  /* Leakage fixes of the coupling (Methods, Fluid-filament Interaction): */
  int32_t mdf_iters;       /* multi-direct forcing iterations, 1..64 (0 or 1: the
                              explicit coupling).  The first spreads the node
                              forces F; each further one samples
                              u = (j + F_grid/2)/rho at the node and spreads
                              2 (U_d - u), U_d = (j/rho at the node) + F/2.
                              The tile-binned and the direct transfer; not with
                              SIM_SPLAT_SORTED; sim_backward differentiates it
                              (binned transfer).                               */
  float marker_offset;     /* two-layer broadcast (Methods, Fluid-filament
                              Interaction): each node acts through two markers
                              at +-marker_offset (cells, <= 1) along its
                              normal (tangent x_next - x_prev; the edge at a
                              chain end), half of its force (and of each MDF
                              correction) at each, and moves with (and MDF
                              samples) the mean of their velocities; density
                              deposit, repulsion and energy stay at the node.
                              The tile-binned and the direct transfer; not
                              with SIM_SPLAT_SORTED; sim_backward
                              differentiates it (binned transfer, with or
                              without MDF).  0: one layer                      */
} sim_params;

/* State and per-node arrays of one world (DEVICE pointers, caller-owned).
 * N = n_particles, F = n_filaments.  Node i of filament f is in
 * [fil_offset[f], fil_offset[f+1]). */
typedef struct sim_arrays {
  int32_t n_filaments, n_particles;
  const int32_t *fil_offset;  /* [F+1] nondecreasing CSR offsets, [0]=0, [F]=N; every
                                 filament has 1..1024 nodes                              */
  int32_t *cell;              /* [2][N] integer part of x (row 0) and y (row 1),
                                 unwrapped (not reduced mod the grid)                    */
  float *frac;                /* [2][N] fractional part in [0, 1); position = cell+frac  */
  const float *rest_angle;    /* [N] rest angle of the joint at interior node i
                                 (between edges i-1 and i); ignored at filament ends     */
  const float *rest_length;   /* [N] rest length of edge (i, i+1); ignored at last node   */
  const float *act_amp;       /* [F] actuation amplitude (rad)                           */
  const float *act_period;    /* [F] actuation period (steps), > 0                        */
  const float *act_phase;     /* [F] actuation phase offset (rad)                        */
  float *f;                   /* [9][ny][nx] pre-collision populations at the current
                                 step, stored SHIFTED by the lattice weights: f_q - w_q.
                                 Velocity order: rest, +x, +y, -x, -y, (+1,+1), (-1,+1),
                                 (-1,-1), (+1,-1).                                        */
  float *u;                   /* [ny][nx][2] out: fluid velocity (x, y interleaved) of
                                 the last step taken                                     */
  /* Optional per-edge parameters and topology (Methods, Filaments: stiffness
   * coefficients on the edge level; filaments with loops).  NULL: the
   * scalars of sim_params, and open chains. */
  const float *k_bend;        /* [N] bending stiffness of the joint at node i            */
  const float *k_stretch;     /* [N] stretch stiffness of the edge leaving node i        */
  const float *k_shear;       /* [N] shear blend of the edge leaving node i              */
  const int32_t *fil_flags;   /* [F] SIM_FIL_CLOSED: filament f is a closed loop (at
                                 least 3 nodes): its last node's edge joins it to the
                                 first (rest_length of the last node), every node is a
                                 joint (the first between the closing edge and edge 0),
                                 and the actuation wave runs over all n joints          */
  /* Optional energy field (Methods, Fields: persistent scalar field of Gaussian
   * packets; Experiments, Neuroevolution: nodes sense the energy at their
   * position, fitness adds the energy collected).  Used when
   * sim_params.energy_rate > 0 and `energy` is given: at every step each node
   * senses e = sum_c W(c - x) E_c at the step's starting position (the
   * transfer kernel), collects energy_rate * e, and the field loses exactly
   * that through the same kernel.  The field does not act on the motion. */
  float *energy;              /* [ny][nx] in/out: the persistent field                 */
  float *energy_sensed;       /* [N] out, may be NULL: e of the last step              */
  float *energy_collected;    /* [F] ACCUMULATED, may be NULL: energy collected per
                                 filament (caller zeroes)                              */
  /* Optional branches (Methods, Filaments: loops and branches with a graph
   * representation; Discussion: cactus graphs).  NULL: no filament hangs
   * from another.  Filament f with fil_parent[f] = p >= 0 hangs from node p
   * of an earlier filament of its creature through an attachment edge from
   * p to f's first node c0.  Each iteration of the PBD projection then runs,
   * after the regular colours of the bending pass, Eq. 1 at p (between p's
   * entering edge and the attachment edge) and then at c0 (between the
   * attachment edge and f's edge 0), and after the regular colours of the
   * position pass, Eqs. 2-4 on the attachment edge; these take the scalar
   * stiffnesses of sim_params and are not actuated.  Rules (SIM_E_INVALID
   * otherwise): p lies in an earlier filament, and every filament between
   * that one and f also hangs from a node (a creature is contiguous); p has
   * an entering edge (a node of a loop, or not the first node of a chain);
   * f is not a closed loop; a node carries at most one filament; a
   * creature holds at most 1024 nodes (sim_batch_admit: the batch's pack
   * capacity).  sim_step_noalloc refuses branched worlds. */
  const int32_t *fil_parent;  /* [F] node filament f hangs from, or -1             */
  const float *fil_attach;    /* [3][F] per filament: attachment rest length, rest
                                 angle at p, rest angle at c0 (ignored for
                                 filaments that hang from no node)                  */
} sim_arrays;

enum { SIM_FIL_CLOSED = 1 };

typedef struct sim_world sim_world;
typedef struct sim_batch sim_batch;

/* Fill *p with the defaults (tau 1, Lambda 1/4, k_bend 0.5, k_stretch 1,
 * k_shear 0.5, 4 PBD iterations, k_elastic 0.05, k_repulse 0.1, sigma 1,
 * radius 4, u_max 0.3, flags 0, tile side 32, no energy field, explicit
 * one-layer coupling) for an nx x ny grid. */
void sim_params_default(sim_params *p, int32_t nx, int32_t ny);

/* Bytes of device workspace sim_create needs for a world of this size. */
sim_status sim_workspace_size(const sim_params *p, int32_t n_filaments, int32_t n_particles,
                              size_t *bytes);

/* Create a world over caller arrays.  Reads fil_offset back to the host
 * (synchronous), validates it, lays out the workspace (256-byte aligned
 * pointer, ws_bytes >= sim_workspace_size) and uploads the work tables.
 * The world's time index is set by each sim_step / sim_rollout call. */
sim_status sim_create(const sim_params *p, const sim_arrays *a, void *workspace, size_t ws_bytes,
                      void *stream, sim_world **out);

/* A set of n_worlds worlds with the same parameters, each with its own
 * arrays (arrays: a host array of n_worlds sim_arrays), stepped together in
 * the same kernel launches: for differentiating many small worlds at once
 * (a population of creatures, Experiments: Filament Folding and the search
 * experiments), where one world's kernels would leave the device idle.
 * sim_step, sim_rollout, sim_checkpoint_size, sim_backward_workspace_size,
 * sim_backward, sim_sync, sim_clear_flags and sim_destroy take a set as they
 * take one world, with every world's part of the caller's buffers one after
 * another in world order: checkpoints (each world's segments, world 0
 * first), g_pos and g_pos0 ([2][N_w] per world), g_rest_angle ([N_w] per
 * world).  The test and measurement hooks (sim_debug_*, sim_profile_steps)
 * refuse sets.  Workspace: sim_set_workspace_size; errors as sim_create. */
sim_status sim_set_workspace_size(const sim_params *p, int32_t n_worlds, const sim_arrays *arrays,
                                  size_t *bytes);
sim_status sim_create_set(const sim_params *p, int32_t n_worlds, const sim_arrays *arrays,
                          void *workspace, size_t ws_bytes, void *stream, sim_world **out);

/* One step at time index t (S0-S7).  Positions, f and u are updated in the
 * caller's arrays when the stream reaches the end of the call. */
sim_status sim_step(sim_world *w, int64_t t);

/* n_steps steps starting at time index t0, launched as captured HIP graphs.
 * If ckpt_every > 0, the state (cell, frac, f) before steps t0, t0+k, ...
 * (k = ckpt_every) is stored into ckpt, which must hold
 * sim_checkpoint_size(w, n_steps, ckpt_every) bytes; ckpt may be NULL iff
 * ckpt_every == 0. */
sim_status sim_rollout(sim_world *w, int64_t t0, int32_t n_steps, int32_t ckpt_every, void *ckpt,
                       size_t ckpt_bytes);

sim_status sim_checkpoint_size(const sim_world *w, int32_t n_steps, int32_t ckpt_every,
                               size_t *bytes);

/* Reverse mode of a rollout (the paper differentiates end to end through the
 * PBD solver and the fluid, Experiments, Filament Folding).  Given the
 * checkpoints written by sim_rollout(t0, n_steps, ckpt_every) and g_pos =
 * dL/dx at the final step ([2][N] device floats), ACCUMULATES dL/d(rest_angle)
 * into g_rest_angle ([N], caller zeroes) and, if g_pos0 is not NULL, WRITES
 * dL/dx at t0 into g_pos0 ([2][N]): chains, closed loops and branched
 * creatures (whose attachment rest lengths and angles are constants).  Each
 * segment is recomputed forward from its checkpoint into adj_ws, then hand-written adjoint kernels run step by
 * step in reverse.  adj_ws must hold sim_backward_workspace_size bytes.
 * The world's own state arrays are not modified.  Only worlds that use the
 * tile-binned transfer (flags without SIM_SPLAT_SORTED / SIM_SPLAT_DIRECT)
 * can be differentiated: for the other two, SIM_E_INVALID is returned before
 * anything is enqueued (their recompute would follow a different summation
 * order than the recorded forward). */
sim_status sim_backward_workspace_size(const sim_world *w, int32_t ckpt_every, size_t *bytes);
sim_status sim_backward(sim_world *w, int64_t t0, int32_t n_steps, int32_t ckpt_every,
                        const void *ckpt, const float *g_pos, float *g_rest_angle, float *g_pos0,
                        void *adj_ws, size_t adj_ws_bytes);

/* Folding objective (Experiments, Filament Folding: mean squared error
 * between the Gaussian-splatted node density at the final step and a target
 * image).  The image covers the periodic nx x ny world: pixel (a, b) of a
 * width x height image is centred at world point
 * (-1/2 + (a + 1/2) nx/width, -1/2 + (b + 1/2) ny/height); every node adds
 * amp * exp(-r^2 / (2 sigma^2)) to each pixel whose centre lies within
 * r <= 5 sigma of it (periodic minimum-image distance).
 *   L = (1 / (width height)) sum_pixels (image - target)^2.
 * The image is summed as 64-bit fixed point (bitwise reproducible). */
typedef struct sim_splat_image {
  int32_t width, height;   /* pixels, 1..16384 each                              */
  float sigma;             /* Gaussian width in cells, > 0                        */
  float amp;               /* peak value of one node's Gaussian                   */
} sim_splat_image;

/* Device workspace bytes sim_density_loss needs for this image. */
sim_status sim_density_loss_workspace_size(const sim_splat_image *img, size_t *bytes);
/* Loss of the nodes at cell + frac ([2][N] device arrays, as in sim_arrays)
 * against target ([height][width] device floats).  Writes *loss (one device
 * float), the image if `image` is not NULL ([height][width] device floats)
 * and dL/dx ([2][N] device floats, overwritten) if `g_pos` is not NULL; feed
 * g_pos to sim_backward for the gradient in the rest angles.  workspace: 256-
 * byte aligned device buffer of sim_density_loss_workspace_size bytes.
 * SIM_E_INVALID if a node's Gaussian would cover more than 65536 pixels. */
sim_status sim_density_loss(const sim_splat_image *img, int32_t nx, int32_t ny, int32_t n_particles,
                            const int32_t *cell, const float *frac, const float *target, float *image,
                            float *loss, float *g_pos, void *workspace, size_t ws_bytes, void *stream);

/* Add Gaussian energy packets to a field ([ny][nx] device floats):
 * field_c += sum_p amps[p] exp(-|c - c_p|^2 / (2 widths[p]^2)), over every cell
 * (minimum-image distance; cell c centred at its integer coordinates).
 * centres [2][P] (x row, y row), amps [P], widths [P]: device arrays. */
sim_status sim_energy_packets(int32_t nx, int32_t ny, int32_t n_packets, const float *centres,
                              const float *amps, const float *widths, float *field, void *stream);

/* Behavioural descriptors of the quality-diversity search (Experiments, QD
 * Search, Eqs. 5-6) for one change of the rest values (a controller writing
 * new rest angles and lengths between steps): per filament f,
 *   effort[f]     += sum over its joints of (old - new rest angle)^2  (E_bend)
 *   effort[F + f] += sum over its edges  of (old - new rest length)^2 (E_pos)
 * with joints and edges as in sim_arrays (fil_flags may be NULL: all open
 * chains).  All arrays are device arrays; effort [2][F] is accumulated
 * (caller zeroes).  Sums are formed in a fixed order (reproducible). */
sim_status sim_rest_effort(int32_t n_filaments, const int32_t *fil_offset, const int32_t *fil_flags,
                           const float *old_rest_angle, const float *new_rest_angle,
                           const float *old_rest_length, const float *new_rest_length, float *effort,
                           void *stream);

/* Wait for the world's stream; report asynchronous HIP errors, the sticky
 * Mach/NaN flag (SIM_E_UNSTABLE), and SIM_E_STATE if the tile bins did not
 * match the positions (a node found its bin full, or the bin counts did not
 * add up to the node count), which only happens when sub-steps are run out
 * of order. */
sim_status sim_sync(sim_world *w);
/* Clear the sticky Mach/NaN flag (enqueued on the stream). */
sim_status sim_clear_flags(sim_world *w);
/* Release host-side resources (graphs, pinned staging).  Does not touch the
 * caller's device memory. */
void sim_destroy(sim_world *w);
const char *sim_last_error(void);

/* For callers that cannot allocate memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): one step at time
 * index t of the world given by *p and *a, with no world handle and no
 * allocation of any kind.  It runs the kernels sim_create + sim_step run and
 * gives the same result; its workspace (work tables, descriptors, per-step
 * buffers) is a static 32 MiB device array of the library, one per device,
 * held until the process ends (enough for a 512 x 512 grid with 65,536
 * nodes).  Everything is enqueued on `stream`, which must belong to the
 * current device; nothing is read back or synchronised.
 *   p, a    as for sim_create (device arrays, caller-owned); positions, f and
 *           u are updated in place when the stream reaches the end of the
 *           call.  Every filament gets a block of its own (up to 1024 nodes).
 *   status  optional DEVICE int32: receives SIM_OK, SIM_E_INVALID (the
 *           filament offsets failed their checks: nothing was changed),
 *           SIM_E_UNSTABLE (NaN or |u| > u_max) or SIM_E_STATE, written at
 *           the end of the step.  May be NULL.
 * Returns SIM_E_INVALID for bad parameters or arrays and SIM_E_WORKSPACE when
 * the world needs more than the static array holds, both before anything is
 * enqueued.  All calls on one device share its array: calls whose work
 * overlaps on the device (different streams, or host threads) race and give
 * undefined results; calls on one stream are ordered and safe. */
sim_status sim_step_noalloc(const sim_params *p, const sim_arrays *a, int64_t t, int32_t *status, void *stream);

/* Test hook: run a single sub-step kernel of step t on the current state
 * (which: 0 elastic force + deposit, 1 filter, 2 repulsion + spread,
 * 3 fluid update, 4 gather + integrate), and expose the world's internal
 * per-step buffers (which: 0 deposit s [ny][nx], SIM_SPLAT_DIRECT only, else
 * NULL; 1 central difference of the filtered density [ny][nx][2]; 2 grid
 * force [ny][nx][2]; 3 total node force [2][N]; 4 elastic node force
 * [2][N]).  For parity tests.  The
 * sub-steps of one step must be run in order, starting with 0. */
sim_status sim_debug_substep(sim_world *w, int32_t which, int64_t t);
/* Test hook: one linear sub-step of the hand-written adjoint on the world's
 * current state, for transpose (dot-product) tests against the forward
 * sub-steps: which 0: out [ny][nx][2] = spread of the node vector in [2][N]
 * (the transpose of the velocity gather; binned worlds, after sub-step 0 of
 * the step); 1: out [ny][nx] = the Gaussian filter applied to the transpose of
 * the central difference of in [ny][nx][2]; 2: out [9][ny][nx] = the
 * transposed Jacobian of the fluid update (collision and streaming, at the
 * world's populations and grid force) applied to in [9][ny][nx]; scratch: 16
 * bytes per cell.  Device pointers; enqueued on the world's stream. */
sim_status sim_debug_adjoint(sim_world *w, int32_t which, const void *in, void *out, void *scratch);
sim_status sim_debug_buffer(sim_world *w, int32_t which, void **ptr);

/* Measurement hook: run n_steps ordinary steps from time index t0 (kernels
 * launched directly, not from a graph) with HIP events on the world's stream
 * around every kernel group, and write the mean device time in milliseconds
 * of each group to ms_out[6]: 0 elastic force, 1 transfer preparation
 * (sorting; the tile bins are built by groups 0 and 5), 2 deposit + filter,
 * 3 repulsion + spread, 4 fluid update, 5 gather + integrate.  Group 4 is the
 * fluid kernel's own execution time (its dispatch's start and end
 * timestamps); the other groups are event pairs around their launches and
 * include dispatch gaps.  The state advances exactly as with sim_rollout.
 * Synchronises the stream. */
sim_status sim_profile_steps(sim_world *w, int64_t t0, int32_t n_steps, float *ms_out);

/* Measurement hook: throughput of the atomic adds a particle -> grid transfer
 * can be built on, on the current device.  buf is a caller DEVICE buffer of
 * at least 64 MiB (256-byte aligned), overwritten.  Writes out[7]: lane
 * operations per clock per compute unit of LDS adds, bank-conflict free,
 * 1024 words per block, 8 blocks of 256 threads per compute unit:
 *   out[0] float add whose result is used, out[1] float add (result unused),
 *   out[2] 64-bit integer add, out[3] 32-bit integer add;
 * out[4] global float atomic adds per clock, whole chip, at scattered words
 * of buf; out[5] the clock (Hz) the rates are counted in (the device's
 * reported peak engine clock); out[6] the compute-unit count.  Each figure is
 * the mean of 5 launches after one warm-up.  Synchronises the stream. */
sim_status sim_measure_atomics(void *buf, size_t buf_bytes, void *stream, double *out);


/* ---- Batched worlds: many independent worlds of uneven size advanced by the
 * same kernels in one persistent, graph-captured launch per chunk of steps.
 * World state lives in a caller-provided device pool (the HBM budget). ---- */

/* Pool bytes one world of this size occupies inside a batch pool. */
sim_status sim_batch_world_bytes(const sim_params *p, int32_t n_filaments, int32_t n_particles,
                                 size_t *bytes);
/* max_worlds slots; pool is a device buffer of pool_bytes (256-byte aligned). */
sim_status sim_batch_create(int32_t max_worlds, void *pool, size_t pool_bytes, void *stream,
                            sim_batch **out);
/* Copy a world's initial state (device arrays in *init) into the pool and
 * give it slot *slot.  It will run `steps` steps from time index t0 and then
 * idle.  SIM_E_FULL: no free slot; SIM_E_WORKSPACE: pool exhausted. */
sim_status sim_batch_admit(sim_batch *b, const sim_params *p, const sim_arrays *init, int64_t t0,
                           int32_t steps, int32_t *slot);
/* Advance every resident world by up to n_steps steps (worlds whose step
 * budget runs out idle); one graph launch per chunk. */
sim_status sim_batch_advance(sim_batch *b, int32_t n_steps);
/* Steps still to run for a slot (host bookkeeping, no sync). */
sim_status sim_batch_remaining(const sim_batch *b, int32_t slot, int32_t *remaining);
/* Copy a slot's state (cell, frac, f, u) into caller arrays *out (same sizes
 * as at admission; enqueued on the stream, then synchronised) and free it.
 * Returns SIM_E_UNSTABLE (and still frees) if that world was flagged. */
sim_status sim_batch_retire(sim_batch *b, int32_t slot, const sim_arrays *out);
sim_status sim_batch_sync(sim_batch *b);
/* Tunables chosen by the autotuner: steps per captured chunk and the
 * persistent grid size (blocks) of the cell and node kernels. */
sim_status sim_batch_set_tuning(sim_batch *b, int32_t chunk_steps, int32_t cell_blocks,
                                int32_t node_blocks);
void sim_batch_destroy(sim_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* MICROCOSM_H */
