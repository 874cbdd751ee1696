/*
 * pic.h -- C ABI of the MI355X (gfx950) implementation of the particle-in-cell
 * pair-potential cycle of Mitchell, Schumacher and Chowdhury, "Modeling crater
 * formation in femtosecond-pulse laser damage from basic principles"
 * (arXiv 1502.07722).
 *
 * The method (the paper's PIC cycle, Fig. 1 and eqs. (1)-(3)):
 *   1. deposit   every macroparticle's weight (number of real atoms it stands
 *                for) onto the nodes around it -> node density;
 *   2. gradient  the density gradient at the half-node (cell-centred) points;
 *   3. gather    node density and centre gradient interpolated back to each
 *                macroparticle with the same linear shape;
 *   4. geometry  mean spacing rbar = n^(-1/3), its gradient by eq. (1), and the
 *                distances to the two nearest neighbours per axis by eq. (2)
 *                (cubic lattice, the paper's assumption);
 *   5. force     pair force from the altered Lennard-Jones potential, eq. (3):
 *                repulsive branch (r < r0) scaled by s_rep, attractive branch
 *                (r >= r0) by the correction factor c_att;
 *   6. push      leapfrog; in 2D positions have two components and velocities
 *                three (the paper's 2D PIC).
 *
 * Conventions shared by every entry point
 *   - Cells are numbered cell = i + n[0]*(j + n[1]*k).  A position is the cell
 *     plus an in-cell offset off[d] in [0, 1) per evolved axis.
 *   - Nodes sit at integer coordinates.  A periodic axis has n[d] nodes, a
 *     reflecting axis n[d] + 1 (wall nodes count half a cell volume each).
 *     node = a0 + nn0*(a1 + nn1*a2), nn_d the node count per axis.
 *   - Weights are fixed point: wq = round(w * 2^20), w in atoms, 0 <= wq < 2^31.
 *   - Deposits are int64 fixed-point sums (offsets quantised to 16 bits, the
 *     weight split axis by axis with the remainder to the lower node), so node
 *     sums are exact and independent of summation order.
 *   - Velocities are half-step (leapfrog) velocities v(n - 1/2) between calls.
 *   - SI units: metres, seconds, kilograms, joules; forces in newtons per atom.
 *   - Particle arrays are structure-of-arrays: off is [ndim][n] (axis-major),
 *     vel is [3][n].
 *
 * Memory and streams
 *   - Every device buffer is owned by the caller (device pointers).  The
 *     library never allocates device memory: pic_init binds a caller-provided
 *     device workspace of at least pic_workspace_bytes() bytes and a HIP
 *     stream; all work is enqueued on that stream.
 *   - Calls are stream-ordered and asynchronous unless stated otherwise.
 *     pic_step and pic_sync synchronise the stream before returning.
 *
 * Errors
 *   - Every function returns an int status (PIC_OK = 0).  No exception ever
 *     crosses the ABI.  pic_last_error(ctx) describes the last failure.
 *   - Argument problems are found on the host before any work is enqueued.
 *   - Problems found on the device (a particle outside the grid or with an
 *     offset outside [0, 1), a negative weight, a step of one cell or more)
 *     set a device error word; that word is read and cleared by pic_step and
 *     pic_sync, which then return the matching code.  Invalid particles are
 *     skipped by the kernels, never used to index memory.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_OK 0
#define PIC_EINVAL 1    /* null pointer, bad dimension, size or parameter */
#define PIC_ERANGE 2    /* cell outside the grid or offset outside [0, 1) */
#define PIC_ECFL 3      /* a particle moved one cell or more in one step */
#define PIC_EOVERFLOW 4 /* negative fixed-point weight */
#define PIC_EHIP 5      /* a HIP runtime call failed */
#define PIC_ENOSPACE 6  /* workspace too small, or n above the bound max_n */

/* Grid of cells and nodes (the paper's partial discretisation, Fig. 1A). */
typedef struct pic_grid {
  int32_t ndim;    /* 2 or 3 */
  int32_t n[3];    /* cells per axis (n[2] ignored in 2D); product < 2^31 */
  double h[3];     /* cell edge per axis, m */
  int32_t bc[3];   /* per axis: 0 periodic, 1 reflecting walls */
  double depth2d;  /* 2D only: thickness the plane stands for, m; <= 0 means h[0] */
} pic_grid_t;

/* Altered pair potential plus the two guards the method needs where eq. (2)
 * stops describing a lattice.  The pair potential U is the paper's
 * Lennard-Jones eq. (3), or the Morse potential, which the paper names among
 * the potentials its density-to-distance map works with:
 *   PIC_POT_LJ     U(r) = D ((r0/r)^12 - 2 (r0/r)^6)
 *   PIC_POT_MORSE  U(r) = D (e^2 - 2e),  e = exp(-alpha (r - r0))
 * Both have their minimum -D at r0 (U'(r0) = 0), where the two branch
 * multipliers switch.
 * The assumed lattice (method section: the paper takes a cubic lattice and
 * notes the construction adapts to hexagonal close packing):
 *   PIC_LATTICE_CUBIC  one neighbour pair per evolved axis, eqs. (1)-(2);
 *   PIC_LATTICE_HCP    the 12 neighbours of an ideal HCP crystal, c axis on
 *                      the normal (last) axis, a basal axis on x, at
 *                      d = 2^(1/6) rbar / (1 - q/2), q = 2^(1/6) grad(rbar).u
 *                      clamped to +-g_clamp (eq. (2)'s midpoint rule along
 *                      each neighbour direction u); force = sum of phi'(d) u.
 *                      In 2D the unresolved basal axis carries no gradient and
 *                      its force component is dropped.  Solid density sits at
 *                      the potential minimum when r0 = 2^(1/6) n_solid^(-1/3).
 * The reverse-mode entry points support both potentials on both lattices. */
#define PIC_POT_LJ 0
#define PIC_POT_MORSE 1
#define PIC_LATTICE_CUBIC 0
#define PIC_LATTICE_HCP 1
typedef struct pic_potential {
  double D;        /* well depth (dissociation energy), J */
  double r0;       /* equilibrium distance, m */
  double s_rep;    /* multiplier on the repulsive branch r < r0 (>= 1) */
  double c_att;    /* multiplier on the attractive branch r >= r0 (> 0) */
  double g_clamp;  /* |d rbar / dx| is clamped to this (0 < g_clamp < 2) */
  double n_floor;  /* no force at densities n <= n_floor, m^-3 */
  double mass;     /* atomic mass, kg */
  int32_t kind;    /* PIC_POT_LJ or PIC_POT_MORSE */
  int32_t lattice; /* PIC_LATTICE_CUBIC or PIC_LATTICE_HCP */
  double alpha;    /* Morse width, 1/m (> 0 for PIC_POT_MORSE; unused otherwise) */
} pic_potential_t;

/* Caller-owned device arrays, structure-of-arrays. */
typedef struct pic_particles {
  int64_t n;       /* number of macroparticles, 0 <= n <= max_n */
  int32_t *cell;   /* [n] linear cell index */
  float *off;      /* [ndim][n] offsets in [0, 1) */
  float *vel;      /* [3][n] half-step velocities, m/s */
  int32_t *wq;     /* [n] weight * 2^20 */
} pic_particles_t;

/* Diagnostics of step n (FP64; the only FP64 arithmetic on the device):
 *   ke   = sum w m/2 (|v(n-1/2)|^2 + |v(n+1/2)|^2)/2          (J)
 *   pe   = sum over nodes V_node eps(n_node)                   (J)
 *          eps: the energy density of the pair potential, eps'(n) = mu(n)
 *   px.. = sum w m (v(n-1/2) + v(n+1/2))/2                      (kg m/s)
 *   wsum = sum w (atoms), bond = sum w (1/2) sum_pairs phi(r)   (J)
 * In 2D, V_node and the energies refer to a slab of thickness depth2d. */
typedef struct pic_diag {
  double ke, pe, px, py, pz, wsum, bond;
  int64_t step;    /* step index within the pic_step call */
} pic_diag_t;

typedef struct pic_ctx pic_ctx_t;

/* Number of nodes of a grid (0 if the grid is invalid). */
int64_t pic_num_nodes(const pic_grid_t *grid);

/* Workspace bytes pic_init needs for this grid and at most max_n particles.
 * Returns 0 if the grid is invalid. */
size_t pic_workspace_bytes(const pic_grid_t *grid, int64_t max_n);

/* Create a context.  Checks the grid and potential, converts them to the
 * kernels' reduced units (length r0, energy D), and binds the caller's device
 * workspace (ws, ws_bytes; 256-byte aligned; must stay valid until
 * pic_destroy) and HIP stream (hipStream_t, NULL = default stream).
 * dt is the time step in seconds.  On failure *out is NULL. */
int pic_init(pic_ctx_t **out, const pic_grid_t *grid, const pic_potential_t *pot, double dt,
             int64_t max_n, void *ws, size_t ws_bytes, void *stream);

/* Free the host-side context (never the caller's device memory). */
int pic_destroy(pic_ctx_t *ctx);

/* Text of the last error on this context (never NULL). */
const char *pic_last_error(const pic_ctx_t *ctx);

/* Wait for the bound stream, then read and clear the device error word. */
int pic_sync(pic_ctx_t *ctx);

/* Step 1: overwrite node_w[pic_num_nodes] with the int64 fixed-point node
 * sums of the particles' weights.  Bit-exact and order independent. */
int pic_deposit(pic_ctx_t *ctx, const pic_particles_t *p, int64_t *node_w);

/* Steps 2-5: per-atom force [ndim][n] (newtons) on every particle from the
 * node sums node_w (as written by pic_deposit).  If pe_or_null is not NULL it
 * receives the grid potential energy (pe field only; synchronises). */
int pic_force(pic_ctx_t *ctx, const pic_particles_t *p, const int64_t *node_w, float *force,
              pic_diag_t *pe_or_null);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): steps 1-5,
 * pic_deposit followed by pic_force, for one grid without a context and
 * without allocating anything.  The node sums, node densities, cell-centred
 * gradients and the device error word live in one static device array of
 * PIC_NOALLOC_SCRATCH_BYTES (64 MiB), which each GPU the library runs on holds
 * until the process ends (pic_init, or else the first call on a device, looks
 * its address up).  Limit: 12 bytes per node plus 4 ndim bytes per cell must
 * fit in it (2D grids up to about 3.3 million cells, 3D up to about 2.7
 * million); larger grids return PIC_ENOSPACE.
 * Runs on the current device, enqueued on stream (hipStream_t, NULL = the
 * default stream of that device), stream-ordered and asynchronous.  Results
 * are bit-identical to pic_deposit and pic_force on a context of the same
 * grid and potential.
 * In:  grid and pot as for pic_init; p: device arrays (cell, off, wq; vel is
 *      not read).
 * Out: force [ndim][n], N per atom (device, caller-owned).  device_error
 *      (device word, may be NULL): invalid particles are skipped, and bit 1
 *      (a cell outside the grid or an offset outside [0, 1)) or bit 4 (a
 *      negative weight) is OR-ed into it; the caller clears it.
 * Returns PIC_EINVAL for NULL or invalid arguments, PIC_ENOSPACE as above,
 * PIC_EHIP if a launch fails.  Every call on a GPU shares that GPU's array:
 * calls that overlap (other streams or threads) race and must be serialised
 * by the caller. */
#define PIC_NOALLOC_SCRATCH_BYTES (64u << 20)
int pic_force_noalloc(const pic_grid_t *grid, const pic_potential_t *pot, const pic_particles_t *p, float *force,
                      uint32_t *device_error, void *stream);

/* v += frac * force / m * dt on the evolved components (frac = -1/2 turns
 * initial velocities v(0) into the half-step velocities v(-1/2)). */
int pic_kick(pic_ctx_t *ctx, pic_particles_t *p, const float *force, double frac);

/* Step 6: one leapfrog push with the given force, in place: kick, drift,
 * carry whole cells, wrap periodic axes, mirror at reflecting walls. */
int pic_push(pic_ctx_t *ctx, pic_particles_t *p, const float *force);

/* nsteps full cycles (steps 1-6) in place.  The particle order of the arrays
 * is preserved.  If diag is not NULL it receives one entry per step whose
 * index (within this call) is a multiple of diag_every (ceil(nsteps /
 * diag_every) entries, host memory).  Synchronises before returning and
 * reports device errors.  Results are bit-identical to nsteps rounds of
 * pic_deposit, pic_force and pic_push. */
int pic_step(pic_ctx_t *ctx, pic_particles_t *p, int32_t nsteps, pic_diag_t *diag,
             int32_t diag_every);

/* Tuning of the tiled pic_step (results do not depend on it: node sums are
 * exact integers and every particle is updated from its own state):
 *   tile        tile edge in cells, a power of two (2D 8..32, 3D 4..8);
 *   halo        cells a particle may drift out of its tile between binnings
 *               before it takes the slower global path (1..4);
 *   chunk       most particles per work item (512..32768);
 *   sort_every  re-bin particles by tile every this many steps; 0 = never;
 *               -1 = adaptive (default): every 48 steps the drifter count of
 *               the previous check is read back without stalling, and the
 *               particles are re-binned once more than n/2048 have drifted
 *               out of their tile window, or after 1024 steps.
 * Grids with more than 65536 x 32768 (2D) or 2048 x 2048 x 512 (3D) cells,
 * or max_n >= 2^30, use the untiled kernels and reject this call.  A tiling
 * whose window (tile + 2 halo + 3 nodes) is longer than a periodic axis is
 * rejected too. */
int pic_set_tiling(pic_ctx_t *ctx, int32_t tile, int32_t halo, int32_t chunk, int32_t sort_every);

/* pic_set_tiling with tiles that are shorter along the last axis (y in 2D, z
 * in 3D): tile cells along every other axis, tile_last cells along the last,
 * a power of two from the smallest tile edge (2D 8, 3D 4) up to tile.  A
 * flatter 3D tile has a smaller window in LDS, so more blocks share a CU.
 * pic_set_tiling(ctx, t, ...) is pic_set_tile_shape(ctx, t, t, ...).  Same
 * checks and errors as pic_set_tiling; on an error the previous tiling is
 * kept. */
int pic_set_tile_shape(pic_ctx_t *ctx, int32_t tile, int32_t tile_last, int32_t halo, int32_t chunk,
                       int32_t sort_every);

/* 1: make pic_step use the untiled kernels (separate deposit, grid pass and
 * gather+force+push launches per step); 0: the tiled fused step (default). */
int pic_set_path(pic_ctx_t *ctx, int32_t untiled);

/* Copy the node sums of the final positions of the last tiled pic_step (as
 * its fused kernel deposited them) into node_w (pic_num_nodes entries; for a
 * batch, every slab's nodes one after another). */
int pic_step_nodes(pic_ctx_t *ctx, int64_t *node_w);

/* Per-phase device time of pic_step, measured with HIP events recorded on
 * the bound stream around each launch (only while timing is on).
 * Phases: 0 deposit (incl. clearing the node sums), 1 density and gradient
 * grid pass, 2 gather+force+push (the dominant kernel: in the tiled step the
 * fused kernel), 3 re-binning by tile, 4 diagnostics reductions, 5 import of
 * the caller's arrays into the binned store and export back, 6 unused (the
 * tiled step advances particles outside their tile window inside its fused
 * kernel, at the end of each work item), 7 graph replays (blocks of 6 steps; graphs are not used while timing is on, so
 * the per-kernel phases above are measured launch by launch). */
#define PIC_NPHASES 8
typedef struct pic_timing {
  double ms[PIC_NPHASES];        /* summed kernel time per phase, ms */
  int64_t launches[PIC_NPHASES]; /* timed launches per phase */
  int64_t drifters_last;         /* drifters in the last step of the last tiled pic_step */
  int64_t items_last;            /* work items of that step */
} pic_timing_t;

/* Turn event timing of pic_step on (1) or off (0); turning it on clears the
 * accumulated figures.  Timing adds a host-side event harvest every few
 * hundred launches; leave it off for plain runs. */
int pic_set_timing(pic_ctx_t *ctx, int32_t on);

/* Accumulated per-phase times since timing was turned on (synchronises). */
int pic_get_timing(pic_ctx_t *ctx, pic_timing_t *out);

/* ---------------------------------------------------------------------------
 * Batches: several independent slabs (e.g. one per absorbed fluence of a
 * damage-threshold sweep) advanced together.  Every step of every slab is one
 * persistent launch of the fused kernel (drifters included); steady
 * stretches of steps are replayed from a captured HIP graph.  Each slab's
 * result is bit-identical to advancing it alone.
 * ------------------------------------------------------------------------- */

/* Workspace bytes for nslab grids (all 2D or all 3D) holding at most max_n[k]
 * particles each; 0 if a grid is invalid or the batch cannot be tiled. */
size_t pic_workspace_bytes_batch(const pic_grid_t *grids, int32_t nslab, const int64_t *max_n);

/* Create a context over nslab slabs sharing one potential and time step.  A
 * batched context supports pic_step_batch, tiling, graph and timing calls;
 * the single-slab calls (pic_deposit, pic_force, pic_kick, pic_push,
 * pic_step) return PIC_EINVAL on it. */
int pic_init_batch(pic_ctx_t **out, const pic_grid_t *grids, int32_t nslab, const pic_potential_t *pot,
                   double dt, const int64_t *max_n, void *ws, size_t ws_bytes, void *stream);

/* nsteps cycles of every slab; parts[k] are slab k's arrays (order kept).
 * diag (optional, host) is [nslab][ceil(nsteps / diag_every)].  Synchronises
 * and reports device errors like pic_step. */
int pic_step_batch(pic_ctx_t *ctx, pic_particles_t *parts, int32_t nsteps, pic_diag_t *diag,
                   int32_t diag_every);

/* Current tiling (any output pointer may be NULL); tile is the edge along
 * every axis but the last. */
int pic_get_tiling(pic_ctx_t *ctx, int32_t *tile, int32_t *halo, int32_t *chunk, int32_t *sort_every);

/* Current tile edges: along every axis but the last, and along the last
 * (either pointer may be NULL). */
int pic_get_tile_shape(pic_ctx_t *ctx, int32_t *tile, int32_t *tile_last);

/* 1 (default): replay blocks of 6 plain steps (no diagnostics, no re-binning
 * decision) from captured HIP graphs; 0: launch every step.  Graphs are only
 * captured on a context bound to a created stream (never the NULL stream). */
int pic_set_graph(pic_ctx_t *ctx, int32_t on);

/* Autotuner: probes tile shape x chunk candidates (square tiles of 8, 16, 32
 * cells in 2D; 4^3, 8^3 and 8 x 8 x 4 cells in 3D; chunk 512 to 16384, plus
 * chunks whose work items fill whole rounds of the persistent grid; halo 2 in
 * 2D, 1 in 3D; re-binning policy
 * unchanged) on the caller's particles for probe_steps steps each, launched
 * step by step (no graph capture inside a probe), timed with events, and
 * keeps the fastest tiling; among the tilings within 1 % of the fastest it
 * takes the one with the largest chunk (the forward steps cannot tell them
 * apart; a reverse sweep pays per work item).  Tune on a state that has run a few steps: a
 * freshly loaded lattice puts exactly the same number of particles in every
 * tile, so a chunk equal to that number looks as good as a larger one until
 * the first moves split half the tiles into two items.  The
 * particles are copied into the internal store for every probe: the caller's
 * arrays are only read.  Results never depend on the tiling. */
typedef struct pic_tuning {
  int32_t tile, halo, chunk;
  int32_t candidates;   /* tilings that were timed */
  double ms_per_step;   /* the kept tiling's probe, ms per step */
  int32_t tile_last;    /* the kept tile edge along the last axis */
} pic_tuning_t;
int pic_autotune(pic_ctx_t *ctx, const pic_particles_t *parts, int32_t probe_steps, pic_tuning_t *out);

/* Host-side calibration of the attractive correction factor: a flat slab of
 * density n_solid (slab_layers cells thick) in a grid with this grid's cell
 * size, a zero-weight atom moved out along the normal (last) axis with unit
 * attractive multiplier; W = -integral of its normal force from the
 * outermost repulsive-to-attractive sign change to infinity; c_att = D / W.
 * Pure host computation, no context needed. */
int pic_calibrate_catt(const pic_grid_t *grid, const pic_potential_t *pot, double n_solid,
                       int32_t slab_layers, double *c_att, double *work);

/* ---------------------------------------------------------------------------
 * Reverse mode (adjoint) of the cycle above, for gradients of a functional J
 * of the final state with respect to the potential parameters and the
 * initial state.  The paper gives no derivatives: these are the exact
 * derivatives of steps 1-6 as implemented, with the fixed-point deposit
 * differentiated as the plain linear (CIC) deposit it approximates to 2^-16
 * cells, the clamp of eq. (1)'s gradient and the density floor with zero
 * derivative where they act, and the branch switch of eq. (3) at r = r0
 * (where U' = 0) taken from the side the forward pass took.
 *
 * Cotangents (device arrays, float, same particle order as the state):
 *   lam_x  [ndim][n]  dJ/d(offset): per cell of displacement along each axis;
 *   lam_v  [3][n]     dJ/dv, s/m;
 *   nbar   [nodes]    dJ/d(n r0^3): cotangent of the node density in units of
 *                     r0^-3;
 *   dtheta [5]        device doubles, ACCUMULATED (+=): dJ/dD (1/J), dJ/dr0
 *                     (1/m), dJ/ds_rep, dJ/dc_att, dJ/dalpha (m; the Morse
 *                     width, PIC_POT_MORSE only: slot 4 gets +0 under
 *                     Lennard-Jones).  The derivatives in D, r0 and alpha
 *                     hold the other parameters, c_att among them, fixed.
 * Both pair potentials (any pair potential enters eq. (3) through U' alone)
 * and both neighbour geometries (cubic, hexagonal close-packed).
 * Single-slab contexts only.  Stream-ordered and asynchronous; device errors
 * (invalid particles) are reported by the next pic_sync or pic_step.
 * Scatters to nodes use float atomics, so nbar, lam_x and dtheta carry
 * FP32 summation-order noise (the forward path stays bit-exact).
 * ------------------------------------------------------------------------- */

/* One reverse leapfrog step.  state holds x(n) and v(n - 1/2) (the state
 * before forward step n), node_w its node sums (pic_deposit of state).
 * In:  lam_x = dJ/dx(n+1) without the deposit term of step n+1,
 *      nbar_next = nbar of step n+1 (NULL when J does not depend on the
 *      densities of step n+1, e.g. the last step), lam_v = dJ/dv(n + 1/2).
 * Out: lam_x = dJ/dx(n) without the deposit term of step n, lam_v =
 *      dJ/dv(n - 1/2), nbar = nbar of step n (overwritten), dtheta += the
 *      parameter terms of step n.
 * The particle's forward step is recomputed from state and node_w (same bits
 * as pic_push), including which walls mirror it.  After the last reverse
 * step, pic_deposit_vjp completes lam_x of the initial state. */
int pic_adjoint_step(pic_ctx_t *ctx, const pic_particles_t *state, const int64_t *node_w, const float *nbar_next,
                     float *lam_x, float *lam_v, float *nbar, double *dtheta);

/* VJP of steps 2-5 (pic_force) at state with node sums node_w:
 * force_bar [ndim][n] = dJ/dF (1/N per atom) ->
 * lam_x += the gather terms, nbar = the node-density cotangent (overwritten;
 * add its deposit term with pic_deposit_vjp), dtheta += parameter terms. */
int pic_force_vjp(pic_ctx_t *ctx, const pic_particles_t *state, const int64_t *node_w, const float *force_bar,
                  float *lam_x, float *nbar, double *dtheta);

/* VJP of step 1 with respect to the positions: lam_x += w * sum over the
 * particle's 2^ndim nodes of nbar * d(density share)/d(offset). */
int pic_deposit_vjp(pic_ctx_t *ctx, const pic_particles_t *state, const float *nbar, float *lam_x);

/* Recorded trajectories: the checkpointed reverse sweep at full speed.
 *
 * pic_forward_record runs nsteps cycles like pic_step (same bits), keeping
 * the particles in the library's tile-binned order and re-binning only at
 * checkpoints (with sort_every < 0 when too many particles left their tile,
 * with sort_every > 0 at every checkpoint, with 0 never), and copying the
 * state and its binning into record before every step that is a multiple of
 * every (checkpoints).  record is caller-owned device
 * memory of pic_record_bytes() bytes, 256-byte aligned; the final state is
 * written back to p in the caller's order.
 *
 * pic_backward_record then runs the whole reverse sweep for that run: for
 * each checkpoint segment, from the last, it recomputes the segment's states
 * and node sums out of place into scratch (pic_backward_bytes() bytes,
 * caller-owned device memory, 256-byte aligned; a record that keeps every
 * state, pic_set_record_states, has them already) and applies the reverse
 * step of pic_adjoint_step to each, last step first.
 * In:  lam_x [ndim][n] = dJ/d(offset) of the final state, lam_v [3][n] =
 *      dJ/dv(nsteps - 1/2) (caller order; J must not depend on the final
 *      node densities).
 * Out: lam_x = complete dJ/d(offset) of the initial state, lam_v =
 *      dJ/dv(-1/2); dtheta (device, 5 doubles) += dJ/d(D, r0, s_rep, c_att,
 *      alpha).
 * start_kick = f != 0: the recorded run's start velocities came from a kick
 *      v(-1/2) = v(0) + f F(x0) dt / m of its initial state (f = -1/2 is the
 *      leapfrog start, pic_kick with frac f).  Its VJP is folded into the
 *      last reverse step (the same state's force VJP with 1 + f times the
 *      step's force cotangent), so lam_v = dJ/dv(0) and lam_x and dtheta
 *      include the terms through F(x0).  0: no start kick.
 * p supplies the particle count (its arrays are not read).  The context, its
 * tiling, nsteps, every and record must be those of the pic_forward_record
 * call, otherwise PIC_EINVAL.  Single-slab contexts on the tiled path only.
 * Synchronises and reports device errors. */
size_t pic_record_bytes(pic_ctx_t *ctx, int32_t nsteps, int32_t every);
size_t pic_backward_bytes(pic_ctx_t *ctx, int32_t every);

/* all = 1: later records keep every state of the run and the node sums of
 * every step, not only the checkpoints (checkpoints still set where the run
 * may re-bin): pic_forward_record writes each step's output straight into
 * the record, and pic_backward_record recomputes nothing, so the sweep is
 * the reverse steps alone.  The record grows to about nsteps x (16 + 4 ndim)
 * bytes per particle slot plus (nsteps + 2) x 8 bytes per node (pic_record_bytes
 * and pic_backward_bytes report the sizes for the current setting); the
 * gradient is the same up to the order of float atomic sums.  0 (default):
 * checkpoints only.  A record must be replayed under the setting it was
 * written with, otherwise pic_backward_record returns PIC_EINVAL. */
int pic_set_record_states(pic_ctx_t *ctx, int32_t all);
int pic_forward_record(pic_ctx_t *ctx, pic_particles_t *p, int32_t nsteps, int32_t every, void *record,
                       size_t record_bytes);
int pic_backward_record(pic_ctx_t *ctx, const pic_particles_t *p, int32_t nsteps, int32_t every,
                        const void *record, size_t record_bytes, void *scratch, size_t scratch_bytes, float *lam_x,
                        float *lam_v, double *dtheta, double start_kick);

/* ---------------------------------------------------------------------------
 * Crater measurement (results section, Figs. 3-4 and eq. (5)).  The paper
 * shows densities in units of the solid density with nothing below 1 % of
 * it (the thin gas there leaves the crater unchanged), measures the crater's
 * width and depth once the surface has settled, and converts width and beam
 * diameter into a threshold fluence by eq. (5): F_th = F exp(-(Gamma/a)^2).
 * How width and depth are read off the map is this library's reading:
 *   - a column is the line of nodes along the normal (last) axis that share
 *     their lateral indices; its equivalent solid thickness t is the weight
 *     of its nodes at or above the cut-off divided by n_solid times the
 *     column's cross-section (the thickness its atoms would have at solid
 *     density);
 *   - depth = the largest deficit y_s - t, y_s the initial surface height;
 *   - columns with deficit >= depth_min are cratered; the crater diameter
 *     Gamma is their total lateral length (2D) or the diameter of the circle
 *     of their total lateral area (3D); a column on a reflecting lateral wall
 *     counts half (a quarter on two);
 *   - eq. (5) with a the beam diameter at which the fluence falls to 1/e of
 *     its peak (sqrt(2) R for a Gaussian of 1/e^2 radius R).
 * ------------------------------------------------------------------------- */
typedef struct pic_crater_spec {
  double n_solid;    /* solid number density, m^-3: the density unit (> 0) */
  double cut;        /* nodes below cut * n_solid count as empty (>= 0; the paper's figures: 0.01) */
  double depth_min;  /* a column is cratered when its deficit is at least this, m (> 0) */
} pic_crater_spec_t;

typedef struct pic_crater {
  double depth;      /* largest deficit y_s - t over the slab's columns, m */
  double width;      /* crater diameter Gamma, m */
  double t_min;      /* thinnest column's equivalent solid thickness, m */
  double t_max;      /* thickest column's, m */
  double f_th;       /* eq. (5) threshold fluence, J/m^2; 0 without fluence and beam diameter */
  int64_t ncols;     /* cratered columns */
} pic_crater_t;

/* Columns of one grid: the product of the lateral axes' node counts. */
int64_t pic_num_columns(const pic_grid_t *grid);

/* Measure every slab of the context on node sums node_w (device, int64, all
 * slabs' nodes one after another as pic_deposit / pic_step_nodes lay them
 * out).  Host arrays, one entry per slab: y_s (initial surface height along
 * the normal axis, m), fluence (peak absorbed fluence, J/m^2) and beam_d
 * (beam diameter, m), the last two NULL when eq. (5) is not wanted.
 * Device outputs, caller-owned: col_w [sum of pic_num_columns] receives
 * each column's kept weight (int64, weight units; overwritten), rho
 * [nodes] (may be NULL) the density map in units of n_solid with zeros
 * below the cut-off (float: the node sum times a float scale, within 2e-7
 * of the FP64 density), out [nslab] the results.
 * The cut-off decision is the FP64 one, (N 2^-20 / V) / n_solid >= cut
 * with V the node volume; the host turns it into an exact integer bound on
 * the node sum N.  Column sums are exact.  Stream-ordered and asynchronous;
 * PIC_EINVAL for NULL or invalid arguments (also a cut whose bound passes
 * 2^52 weight units).  The kernels read node_w once: a call costs about 8
 * bytes per node (12 with rho) plus 24 per column. */
int pic_crater(pic_ctx_t *ctx, const int64_t *node_w, const pic_crater_spec_t *spec, const double *y_s,
               const double *fluence, const double *beam_d, float *rho, int64_t *col_w, pic_crater_t *out);

/* Threshold fluence over a sweep of n fluences with measured crater
 * diameters (host arrays; slabs with width <= 0 are left out):
 * f_th_fixed = geometric mean of the per-slab eq. (5) values at beam
 * diameter beam_d (the least-squares ln F_th with a held fixed);
 * f_th_fit and beam_d_fit from the least-squares line Gamma^2 = a^2 ln F -
 * a^2 ln F_th.  Outputs are NaN when fewer than one (fixed) or two distinct
 * fluences (fit) remain, or the fitted slope is not positive.  Host only. */
int pic_threshold_fit(int32_t n, const double *fluence, const double *width, double beam_d, double *f_th_fixed,
                      double *f_th_fit, double *beam_d_fit);

#ifdef __cplusplus
}
#endif
#endif /* PIC_H */
