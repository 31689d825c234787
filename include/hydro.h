/*
 * hydro.h -- C ABI of the MI355X (gfx950) Godunov hydrodynamics library.
 *
 * The library advances the Euler equations of a gamma-law gas (eq. hydro of
 * Wang, "The Kratos Framework for Heterogeneous Astrophysical Simulations",
 * arXiv 2501.02317) on a uniform Cartesian mesh with the method of its
 * Sec. 3: primitive-variable PLM reconstruction with the minmod limiter
 * (eq. minmod), the HLLC Riemann solver with subtraction-safe wave speeds
 * (eqs. hllc-contact-spd and hllc-mixed-dvel), a flux-divergence update in
 * the Heun two-stage integrator (Sec. 3.3), and a global CFL time step taken
 * at the first sub-step (Sec. 3.1).  Ghost zones follow Sec. 3.1.1 and are
 * resolved inside the kernels' loads; no ghost layers are stored, except the
 * restricted and prolonged layers at the level jumps of a refined mesh.
 *
 * Data conventions
 *   - ndim in {1,2,3}; n[d] interior cells on axis d; axes d >= ndim must
 *     have n[d] == 1.  ncomp = 2 + ndim.  A plane of the kernels' marching
 *     axis (n[0] * n[1] cells in 3-D, n[0] in 1-D and 2-D) must hold fewer
 *     than 2^29 cells.
 *   - Conserved state U = (rho, m_1..m_ndim, E), primitive W = (rho,
 *     v_1..v_ndim, p): only in-plane momenta are carried.
 *   - Host and device fields are FP64, layout [comp][k][j][i] with i (x)
 *     fastest, interior cells only (ncomp * n[0] * n[1] * n[2] doubles).
 *   - Precision (Sec. 3.2.2): HYDRO_FP64 does everything in FP64.
 *     HYDRO_MIXED converts to primitive variables in FP64, rounds them to
 *     FP32, does PLM and HLLC in FP32, and keeps the flux difference, the
 *     Heun combine, the predictor, dt and the totals in FP64.
 *
 * Memory, streams and threads
 *   - Device memory is owned by the caller: hydro_create carves its state
 *     out of a caller-provided device workspace of at least
 *     hydro_workspace_bytes(cfg) bytes (256-byte aligned), which must outlive
 *     the handle.  The handle itself owns only host metadata (among it a
 *     pageable mirror of its control block) and, once hydro_set_block_streams turns them
 *     on, its block streams and events (a refined handle: its second stream
 *     and three events).  hydro_stage_rhs,
 *     hydro_padded_primitive and the host transfers of a split mesh take a
 *     temporary device buffer (stream-ordered allocation) for the call.
 *   - All device work is enqueued on the caller's HIP stream given at
 *     creation (NULL = the legacy default stream).
 *   - hydro_step / hydro_step_auto return after enqueueing.  hydro_cfl_dt,
 *     hydro_conserved_totals, hydro_time, hydro_get_state and the setters
 *     block until the stream has drained.
 *   - A handle is not thread safe; serialise calls per handle.
 *
 * Errors
 *   Every call returns HYDRO_OK (0) or a negative status; nothing throws or
 *   aborts across the ABI.  Invalid arguments return HYDRO_E_INVAL without
 *   side effects.  A non-physical state met by a kernel (rho <= 0, p <= 0 or
 *   a non-finite value in a stage input) sets a sticky device flag that the
 *   next blocking call reports as HYDRO_E_NONPHYSICAL.  A failed HIP call
 *   returns HYDRO_E_DEVICE; the handle then only accepts hydro_destroy.
 */
#ifndef HYDRO_H
#define HYDRO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hydro_ctx* hydro_t;
typedef struct hydro_batch_ctx* hydro_batch_t;

enum hydro_status {
    HYDRO_OK = 0,
    HYDRO_E_INVAL = -1,
    HYDRO_E_NOMEM = -2,
    HYDRO_E_DEVICE = -3,
    HYDRO_E_NONPHYSICAL = -4,
    HYDRO_E_STATE = -5
};

enum hydro_precision { HYDRO_FP64 = 0, HYDRO_MIXED = 1 };

/* Time integrators (Sec. 3.3).  HYDRO_HEUN: the two-stage Heun method (the
 * default); its predictor U1 is kept in FP64.  HYDRO_VL2: the memory-
 * optimised van Leer integrator: a half-step predictor with piecewise-
 * constant face states, W* = W(U^n + (dt/2) L_1(U^n)), kept only as
 * primitive variables in the compute precision (FP32 in HYDRO_MIXED), then
 * U^{n+1} = U^n + dt L_2(W*) with PLM face states.  The predictor never
 * enters U^{n+1} directly, so conservation still holds to FP64 round-off,
 * and in HYDRO_MIXED the workspace needs 60 instead of 80 bytes per cell in
 * 3-D. */
enum hydro_integrator { HYDRO_HEUN = 0, HYDRO_VL2 = 1 };

/* Boundary rules per axis side (Sec. 3.1.1): periodic (both sides of an
 * axis), free (zero gradient), outflow (free, normal velocity clipped so no
 * fluid enters), reflecting (mirror with the normal velocity negated). */
enum hydro_bc { HYDRO_BC_PERIODIC = 0, HYDRO_BC_FREE = 1, HYDRO_BC_OUTFLOW = 2, HYDRO_BC_REFLECT = 3 };

typedef struct {
    int32_t ndim;      /* 1, 2 or 3 */
    int32_t n[3];      /* interior cells per axis, n[d] = 1 for d >= ndim */
    double lo[3];      /* domain lower corner (active axes) */
    double hi[3];      /* domain upper corner, hi > lo */
    double gamma;      /* adiabatic index, > 1 */
    double cfl;        /* Courant number in (0, 1] */
    int32_t precision; /* enum hydro_precision */
    int32_t bc[3][2];  /* enum hydro_bc per axis side (low, high) */
    int32_t integrator; /* enum hydro_integrator */
    int32_t blocks[3]; /* blocks per axis (0 or 1: one); see "Blocks" below */
} hydro_config;

/*
 * Blocks.  A mesh may be split into blocks[0] x blocks[1] x blocks[2] blocks
 * of equal extents, as the paper's framework splits a domain into blocks of
 * the same size: blocks[d] must divide n[d], a split axis must leave every
 * block at least 2 cells on it, blocks[d] = 1 for d >= ndim, and there are at
 * most 1024 blocks.  The device state is then stored block after block,
 * [block][comp][k][j][i] of the block's extents, with block index
 * b0 + blocks[0] (b1 + blocks[1] b2); every host transfer and
 * hydro_get_state_device / hydro_set_primitive_device still use the mesh
 * layout above, and hydro_state_device returns the block layout.  The faces
 * between blocks are c-boundaries (Sec. 3, block boundaries): a stage reads a
 * block's ghost cells straight from the neighbouring block's cells on the
 * same device, with no ghost storage and no copy; the faces of the whole mesh
 * follow the boundary rules.  Results are bitwise those of the unsplit mesh.
 */

/* Device bytes a handle for cfg needs; 0 when cfg is invalid. */
size_t hydro_workspace_bytes(const hydro_config* cfg);

/* Validate cfg, carve the workspace, and bind the stream.  The state is zero
 * until hydro_set_state / hydro_set_primitive.  *out receives the handle.
 * The zeroing is enqueued on the stream and the call returns without waiting
 * for the stream (work already in flight there is not waited for). */
int hydro_create(const hydro_config* cfg, void* d_workspace, size_t nbytes, void* hip_stream,
                 hydro_t* out);

/* Copy a host conserved state in (layout above) and reset t to 0. */
int hydro_set_state(hydro_t h, const double* U_host);

/* Copy a host primitive state in and convert it to conserved variables on
 * the device (m = rho v, E = p/(gamma-1) + (1/2) sum m v); reset t to 0. */
int hydro_set_primitive(hydro_t h, const double* W_host);

/* As hydro_set_primitive from a device array of the same layout (async;
 * the array must stay valid until the stream reaches this call). */
int hydro_set_primitive_device(hydro_t h, const double* d_W);

/* Copy the current conserved state out (blocks). */
int hydro_get_state(hydro_t h, double* U_host);

/* Copy the current conserved state to a device array (async). */
int hydro_get_state_device(hydro_t h, double* d_U);

/* Device address of the current conserved state (valid until the next step;
 * the block layout when the mesh is split). */
int hydro_state_device(hydro_t h, const double** d_U);

/* CFL step of the current state, cfl * min over cells and active axes of
 * dx_d / (|v_d| + sqrt(gamma p / rho)) (Sec. 3.1).  Blocks. */
int hydro_cfl_dt(hydro_t h, double* dt);

/* One Heun step of length dt > 0 (async): stage 1 U1 = U + L(U) dt, stage 2
 * U = U/2 + (U1 + L(U1) dt)/2, each stage fused into one kernel. */
int hydro_step(hydro_t h, double dt);

/* nsteps Heun steps with the CFL dt kept on the device (async, no host
 * synchronisation).  The dt of each step comes from the previous step's
 * stage-2 epilogue (the first from a standalone reduction).  When t_end > 0
 * the step that would pass t_end is shortened to land on it and later steps
 * are no-ops.
 * hydro_step and hydro_step_auto enqueue kernels only (no allocation, memset
 * or host synchronisation), so a caller may capture them into a HIP graph on
 * the handle's stream.  While that stream is being captured, the forms that
 * fork work onto other streams (block streams, a refined mesh's second
 * stream) run on the handle's stream alone; the results are the same. */
int hydro_step_auto(hydro_t h, int nsteps, double t_end);

/* dV-weighted conserved totals, ncomp values: deterministic compensated
 * FP64 sums in a fixed order (blocks). */
int hydro_conserved_totals(hydro_t h, double* totals);

/* For callers that cannot allocate or synchronise (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): the totals of
 * hydro_conserved_totals for a state the caller holds in device memory,
 * computed with no allocation, no host synchronisation and no memset, and
 * written to device memory.
 *   cfg       the mesh (as for hydro_create; precision and integrator are not
 *             used); its cell volume dV = prod_d (hi_d - lo_d) / n_d.
 *   d_U       device, ncomp * n[0] * n[1] * n[2] doubles, caller-owned: the
 *             layout of hydro_state_device for that configuration (the mesh
 *             layout [comp][k][j][i]; for a split mesh the block layout).
 *   d_totals  device, ncomp doubles, caller-owned: totals_c = dV * sum_i U_c,i,
 *             bitwise the values hydro_conserved_totals returns for a handle
 *             of the same configuration holding the same state.
 *   hip_stream  the work is enqueued there and the call returns at once.
 * Scratch: the partial sums live in a static device array of the library,
 * 2 * 5 * 1024 doubles (80 KiB) per device, which each device holds until
 * the process ends; the reduction never needs more, whatever the mesh size
 * (at most 1024 work-groups of partials; a configuration needing more is
 * refused with HYDRO_E_INVAL).  Calls on one device share that array:
 * calls that overlap on one device (different streams, or threads) race and
 * must be serialised by the caller.  The first call on a device resolves the
 * array's device address (hipGetSymbolAddress), so make it outside a graph
 * capture.  Returns HYDRO_E_INVAL for an invalid cfg or null pointer,
 * HYDRO_E_DEVICE when a HIP call fails; state errors are not checked. */
int hydro_conserved_totals_noalloc(const hydro_config* cfg, const double* d_U, double* d_totals,
                                   void* hip_stream);

/* Run limit kept on the device: device-dt steps (hydro_step_auto, batches)
 * stop advancing this mesh once max_steps more steps are done (0: no step
 * limit) or t reaches t_end (0: no time limit; the last step is shortened to
 * land on it).  Async.  hydro_run_done blocks and reports whether the limit
 * is reached.  hydro_step_auto replaces the time limit with its own and
 * clears the step limit. */
int hydro_set_run_limit(hydro_t h, int64_t max_steps, double t_end);
int hydro_run_done(hydro_t h, int* done);

/* Simulation time and completed step count (blocks). */
int hydro_time(hydro_t h, double* t);
int hydro_steps_done(hydro_t h, int64_t* steps);

/* One stage right-hand side dU = sum_d dt/dx_d (F_{d,i-1/2} - F_{d,i+1/2})
 * of the current state, copied to the host (blocks).  Same kernel as the
 * stages, writing the increment instead of the update. */
int hydro_stage_rhs(hydro_t h, double dt, double* dU_host);

/* Primitive state with the two ghost layers of every active axis resolved
 * by the boundary rules, as the kernels see it (FP64 mode: exact; mixed:
 * the FP32-rounded values), copied to the host in a padded [comp][K][J][I]
 * array with n_d + 4 cells on active axes; corner ghosts are set to 0. */
int hydro_padded_primitive(hydro_t h, double* Wpad_host);

/* Tile of a stage kernel: a work-group covers tx x ty cells of the (x, y)
 * plane (3-D: 32x8, 64x8, 16x16 or 32x16; 1-D and 2-D: 64, 128 or 256 by 1)
 * and marches along the last active axis over chunks of kz planes.  kz = 0
 * (2-D and 3-D) picks the chunk length at each launch so that one round of
 * the work-groups the device holds at once covers the mesh (at least 16 and
 * at most 128 planes; in a batch, about 2048 work-groups per member).  The
 * two stages have a tile each (the stage right-hand side uses stage 1's;
 * a batch uses each member's stage-1 tile for both stages).  Every face flux
 * is the same function of the same inputs for any tile, so the results are
 * bitwise independent of the tiles; only speed changes.  hydro_create picks
 * defaults.  Unsupported shapes or a stage other than 0 (both), 1 or 2 return
 * HYDRO_E_INVAL; hydro_set_tile sets both stages. */
int hydro_set_tile(hydro_t h, int tx, int ty, int kz);
int hydro_set_stage_tile(hydro_t h, int stage, int tx, int ty, int kz);
int hydro_get_stage_tile(hydro_t h, int stage, int* tx, int* ty, int* kz);

/* The tiles the autotuner tries for a configuration: writes up to max
 * (tx, ty, kz) triples to tiles[3 * i ...] and returns their total number
 * (HYDRO_E_INVAL for an invalid configuration or max < 0). */
int hydro_tile_candidates(const hydro_config* cfg, int* tiles, int max);

/* Autotuner.  Advances the run by one untimed step and then steps_per_tile
 * real Heun steps per candidate tile, the candidates taking turns (device-
 * resident dt as in hydro_step_auto, t_end 0 = no clamp), timing each stage
 * with HIP events, and sets each stage's fastest tile; the tile in use is
 * kept unless a candidate beats it by more than 5 %.
 * tiles receives 6 ints (stage 1 tx, ty, kz, then stage 2) and ms_per_step
 * 2 doubles (the chosen tiles' stage times per step).  The steps are part of
 * the run (results do not depend on the tiles), so tuning can replace
 * warm-up steps.  Blocks until done.  If the run reached its limit while
 * tuning (timings of skipped steps mean nothing) the tiles are left as they
 * were and the call returns HYDRO_E_STATE; the handle stays usable.
 * steps_per_tile in [1, 64]. */
int hydro_autotune(hydro_t h, int steps_per_tile, double t_end, int* tiles, double* ms_per_step);

/* Event timing of the stage kernels, for measurement: after
 * hydro_profile(h, cap) the next cap launches of each stage kernel are
 * bracketed by HIP events on the handle's stream (cap = 0 turns timing off
 * and frees the events).  hydro_profile_read blocks, returns the summed
 * durations in milliseconds of the recorded stage-1 and stage-2 launches and
 * their counts (launches[0], launches[1]), and restarts the recording. */
int hydro_profile(hydro_t h, int cap);
int hydro_profile_read(hydro_t h, double* ms_stage1, double* ms_stage2, int64_t* launches);

/*
 * Static mesh refinement (Sec. 2.3: the 2^d-tree of blocks, refined
 * recursively, with face-neighbouring blocks at most one level apart; Sec. 3:
 * c-boundaries across levels).  The blocks of cfg (see "Blocks") are the
 * root blocks of level 0.  refined[] lists nref distinct blocks to refine,
 * each by its code L * 2^26 + (its index on the level-L block grid of
 * blocks[d] 2^L blocks per active axis, x fastest); a root's code is its
 * root index b0 + blocks[0] (b1 + blocks[1] b2).  A block of level L >= 1 can
 * be listed only with its parent, and L <= 2, so leaves reach level 3 at
 * most.  Each listed block is replaced by 2^ndim blocks of half the size and
 * the same extents in cells; then, as the paper does, refinement is added on
 * the coarser side until no two face-neighbouring leaves are more than one
 * level apart.  Refinement needs even block extents of at least 4 cells on
 * the active axes and at most 1024 leaves; both integrators are supported.
 * The van Leer integrator (Sec. 3.3) keeps its predicted state on a refined
 * handle as conserved FP64 values in the second field (not primitive values
 * of the compute type), so the level-jump passes below apply to its
 * predictor (fluxes of piecewise-constant states, half a step) and corrector
 * alike; the workspace is the same for both integrators.
 *   - Leaves are ordered by level, and within a level in the order of that
 *     level's block grid (x fastest).  hydro_smr_leaves writes (level, c0,
 *     c1, c2) per leaf (at most max entries, block coordinates on the leaf's
 *     level, physical axes) and returns the number of leaves, or
 *     HYDRO_E_INVAL; it needs no device.
 *   - A refined handle's host and device state transfers use the block
 *     layout [leaf][comp][k][j][i] of one block's extents (the mesh has no
 *     single uniform layout); its totals weight each level by its cell volume.
 *   - Each stage: the ghost layers at level jumps are filled first, the
 *     coarse side's by volume averages (restriction) of the fine cells, then
 *     the fine side's by minmod-limited prolongation (eq. minmod) of the
 *     coarse cells level by level from the coarsest (a coarse block's
 *     stencil may include its own prolonged layers), on primitive variables, into ghost slots in the
 *     workspace; then the stage kernel runs per level (same-level faces read
 *     the neighbour's cells in place); then each coarse cell next to a level
 *     jump is corrected so that its update uses the mean of the fine fluxes
 *     through its face, which keeps the totals conserved.  One global time
 *     step (the paper's default), taken from a reduction after the step.
 *     The prolongation and the flux recomputation run on a second stream the
 *     handle creates (default priority, non-blocking), overlapping the
 *     level-0 stage; every step joins it back into the handle's stream.
 *   - Not available on a refined handle (HYDRO_E_INVAL): hydro_stage_rhs,
 *     hydro_padded_primitive, hydro_autotune, hydro_set_block_streams(h, 1),
 *     batch membership.
 */
size_t hydro_smr_workspace_bytes(const hydro_config* cfg, int nref, const int32_t* refined);
int hydro_smr_create(const hydro_config* cfg, int nref, const int32_t* refined, void* d_workspace, size_t nbytes,
                     void* hip_stream, hydro_t* out);
int hydro_smr_leaves(const hydro_config* cfg, int nref, const int32_t* refined, int32_t* leaves, int max);

/*
 * How the stages of a split mesh are launched (Sec. 3, Fig. hydro_proc: the
 * blocks' work on streams of their own).  on = 0 (the default): one launch
 * per stage covers every block.  on = 1: the blocks are split into up to four
 * groups of contiguous blocks, each with a stream the handle creates (default
 * priority, not synchronising with the legacy default stream); each group's
 * stage is one launch; a group's stage 2 waits only for the groups that hold
 * its blocks' face neighbours to finish stage 1, and the step's time-step
 * update waits for every group.  The results do not depend on the choice.
 * Stage timing (hydro_profile) records only the one-launch form.  No effect
 * on a mesh of one block.  Blocks until the handle's stream has drained.
 */
int hydro_set_block_streams(hydro_t h, int on);

int hydro_destroy(hydro_t h);

const char* hydro_strerror(int status);

/*
 * Batches: many independent meshes (any mix of ndim, sizes, precision and
 * tiles) advanced together.  The members are existing handles that share one
 * HIP stream; the batch keeps a descriptor table, a work-group table and a
 * member status table in a caller-owned device workspace of hydro_batch_workspace_bytes(n, members)
 * bytes (0 when the members are invalid: NULL, repeated, broken, or on
 * different streams).  A batched step is one launch per (ndim, precision,
 * tile) group for each stage over all members' tiles, then one launch that
 * advances every member's time and device dt; each member keeps its own dt
 * and run limit (hydro_set_run_limit), and members that reached it are
 * skipped.  With use_graph != 0 and a non-default stream, the nsteps-step
 * sequence is captured once into a HIP graph and replayed (recaptured when
 * nsteps changes).  Without a graph, and when the stream is not being
 * captured, a batch of several groups spreads them over its stream and up
 * to two more streams of its own (made at the first such step, freed by
 * hydro_batch_destroy): each group's stages and its members' time / dt
 * update follow one another on one stream, step after step, forked from the
 * members' stream at the call and joined back to it before the call
 * returns, so work enqueued on that stream afterwards sees every step.
 * hydro_batch_step is async; read results through the
 * member handles after synchronising the stream.  Results equal those of
 * stepping each member alone with hydro_step_auto.
 */
size_t hydro_batch_workspace_bytes(int n, const hydro_t* members);
int hydro_batch_create(int n, const hydro_t* members, void* d_workspace, size_t nbytes, int use_graph,
                       hydro_batch_t* out);
int hydro_batch_step(hydro_batch_t b, int nsteps);

/* Batch autotuner.  Tries tile rules for the members of one or two
 * dimensions (a common row width of 64, 128 or 256 cells or each member's
 * own, with each member's own or a fixed chunk length of 16, 32 or 64
 * planes; 3-D members keep their tiles) by timing steps_per_rule batched
 * steps per rule, the rules taking turns after one untimed step, and keeps
 * the fastest rule (the members' own tiles unless beaten by more than 5 %):
 * it becomes the members' tile for both stages.  The steps are real steps of
 * every member (the results do not depend on the tiles) and count against
 * their run limits.  *rule receives the rule index (0: members' own tiles)
 * and *ms_per_step its time per batched step.  Blocks.  steps_per_rule in
 * [1, 64].  The batch workspace (hydro_batch_workspace_bytes) is sized for
 * every rule. */
int hydro_batch_autotune(hydro_batch_t b, int steps_per_rule, int* rule, double* ms_per_step);

/* Per-member run-limit flag (done[i] = 1 once member i reached its limit),
 * optional completed step counts and sticky error flags (bit 0:
 * non-physical state); blocks on the batch stream (one small gather launch
 * and one copy for all members). */
int hydro_batch_status(hydro_batch_t b, int* done, int64_t* steps, int* flags);
/* Number of launch groups, total work-groups per stage, and whether steps run from a graph. */
int hydro_batch_info(hydro_batch_t b, int* groups, int64_t* workgroups, int* graph);
int hydro_batch_destroy(hydro_batch_t b);

/* HLLC fluxes of nfaces face-normal state pairs on the device (async on
 * stream): WL, WR, F are device arrays [ntan+3][nfaces] of FP64 holding
 * (rho, u, t_1..t_ntan, p) and the (mass, normal momentum, tangential
 * momenta, energy) fluxes; precision selects FP64 or FP32 arithmetic.  The
 * same device function the stage kernels use. */
int hydro_riemann_fluxes(int precision, int ntan, double gamma, int64_t nfaces, const double* d_WL,
                         const double* d_WR, double* d_F, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif
