/*
 * mrlbm: multiresolution-adapted lattice Boltzmann hot path for MI355X (gfx950).
 *
 * The method is the adaptive lattice Boltzmann scheme of Bellotti, Gouarin,
 * Graille and Massot (arXiv 2103.02903). One time step follows Algorithm 1
 * ("Overall solver") of the paper:
 *   1. mesh adaptation Lambda(t+dt) = G(H_eps(T_eps(Lambda(t)))) with details of
 *      the current solution (sections "Details and local regularity", "Mesh
 *      coarsening", "Construction of the time adaptive mesh"), followed by the
 *      transfer of the leaf data to the new complete leaves;
 *   2. on every complete leaf, the MR transport of eq. (AdaptiveAdvectionPhase),
 *      evaluated with the flattened weights of eq. (PredictionWithMatrixNew) and
 *      the detail correction next to finer neighbours (section "A non-recursive
 *      implementation of the reconstruction operator");
 *   3. the collision of eq. (AdaptiveCollision) on the same leaf.
 * Each axis is periodic or bounded by walls (section "Boundary conditions"); the
 * prediction stencil half-width is gamma = 1, 2 or 3 (Table 1).
 *
 * Data layout (shared by every host<->device exchange below):
 *   levels l = jmin..jmax are concatenated; level l holds N_l^d cells, N_l = 2^l,
 *   cell index c = x (1D), x + N_l * y (2D) or x + N_l * (y + N_l * z) (3D);
 *   tree    uint8  [level][cell]      1 = the cell belongs to the complete tree;
 *   values  real   [level][h][cell]   real = double (precision 8) or float (4);
 *                                     only complete leaves carry meaningful data.
 *   moments real   [nc][N_J^d]        conserved moments on the finest level:
 *                                     nc = 1 (u) for D1Q2 / D1Q3 / D3Q6,
 *                                     nc = 3 (rho, q_x, q_y) for D2Q9,
 *                                     nc = 4 (rho, rho u, rho v, E) for the Euler scheme.
 *
 * Ownership: the caller allocates the workspace (size from
 * mrlbm_workspace_size) on the device, and owns every input and output buffer.
 * The library never allocates or frees device memory; the context points into
 * the workspace, which must outlive it. All device work is enqueued on the
 * stream given at creation (a hipStream_t); calls that return results to host
 * memory synchronise that stream. A context is not thread-safe.
 *
 * Errors: every function returns a status (0 = OK, < 0 = error, see below);
 * no exception or abort crosses the boundary. After an error the context stays
 * valid for mrlbm_destroy. Device-side failures are sticky flags in the
 * workspace, reported by the next call that synchronises the stream
 * (mrlbm_get_state, mrlbm_get_mesh, mrlbm_stats, mrlbm_leaves, mrlbm_fields):
 * MRLBM_ERR_SYNC if a wait between the two halves of a paired launch ran out
 * of its spin budget (the launch then finished without the ordering, so every
 * later result of the context is invalid until it is destroyed).
 */
#ifndef MRLBM_H
#define MRLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MRLBM_OK 0
#define MRLBM_ERR_INVALID (-1)   /* bad argument or parameter */
#define MRLBM_ERR_CAPACITY (-2)  /* workspace or output buffer too small */
#define MRLBM_ERR_NONFINITE (-3) /* a leaf value is NaN or infinite */
#define MRLBM_ERR_HIP (-4)       /* a HIP runtime call failed */
#define MRLBM_ERR_STATE (-5)     /* call out of order (e.g. step before init) */
#define MRLBM_ERR_SYNC (-6)      /* a device-side wait gave up: the context's results are invalid (sticky) */

#define MRLBM_D1Q2 1 /* linear advection, eta = (+1, -1), m_eq = (u, V u) */
#define MRLBM_D1Q3 2 /* Burgers, eta = (0, +1, -1), m_eq = (u, u^2/2, alpha lambda^2 u) */
#define MRLBM_D2Q9 3 /* Lallemand-Luo MRT of the von Karman section of the paper */
/* Vectorial D2Q4 scheme of the Euler system (section "Systems of hyperbolic
 * conservation laws"): four D2Q4 schemes, one per conserved variable rho,
 * rho u, rho v, E; velocities lambda (1, 0), (0, 1), (-1, 0), (0, -1); moments
 * of variable i: u_i, lambda (f0 - f2), lambda (f1 - f3), lambda^2 (f0 - f1 +
 * f2 - f3), with equilibria u_i, Phi_x,i(u), Phi_y,i(u), 0 and the pressure
 * law p = (gamma_gas - 1) (E - rho (u^2 + v^2) / 2). Population 4 i + k is
 * velocity k of variable i, and so is moment 4 i + k. */
#define MRLBM_D2Q4_EULER 4
/* D3Q6 advection (section "Three dimensional advection equation"): velocities
 * lambda cos(pi h) along x (h = 0, 1), y (h = 2, 3) and z (h = 4, 5); moments
 * u = sum f, lambda (f0 - f1), lambda (f2 - f3), lambda (f4 - f5),
 * lambda^2 (f0 + f1 - f2 - f3), lambda^2 (f0 + f1 - f4 - f5) with equilibria
 * u, V_x u, V_y u, V_z u, 0, 0 (V = mrlbm_params.velocity). Three-dimensional:
 * cell index x + N_l (y + N_l z); periodic boundaries, gamma = 1 and jmax <= 8
 * only; no adjoint. */
#define MRLBM_D3Q6 5

typedef struct mrlbm_ctx mrlbm_ctx;

typedef struct {
  int scheme;      /* MRLBM_D1Q2, MRLBM_D1Q3, MRLBM_D2Q9, MRLBM_D2Q4_EULER or MRLBM_D3Q6 */
  int jmin, jmax;  /* coarsest and finest level: 1 <= jmin <= jmax, jmax <= 8 (3D) / 13 (2D) / 25 (1D) */
  int precision;   /* 8: populations, details and weights in double; 4: in float */
  double lambda;   /* lattice velocity dx/dt (> 0) */
  double eq_param; /* D1Q2: advection velocity V; D1Q3: alpha; D2Q9: ignored; Euler: gamma_gas > 1 */
  double eps;      /* threshold epsilon >= 0 of eq. (Thresholding) */
  double mu_bar;   /* regularity guess in [0, 2 gamma + 1] of the refinement rule */
  double s[16];    /* relaxation rate of each moment (q of them); conserved moments must be 0 */
  /* Boundary of each side x-, x+, y-, y+ (section "Boundary conditions"):
   * MRLBM_PERIODIC, or a wall with the condition of eq. refBoundaryConditions
   * (MRLBM_COPY, MRLBM_BOUNCE_BACK, MRLBM_ANTI_BOUNCE_BACK). An axis is
   * periodic on both sides or walled on both; 1D uses the x sides only. At a
   * wall, the finest cells of the transport sets E beyond it take the side's
   * condition evaluated directly on the leaf (eq. AdvectionOnBoundary, the
   * paper's choice); a cell beyond two walls takes the x wall's condition. The
   * prediction, the details and the reconstruction extend each level by even
   * reflection across a wall, and the mesh's neighbour additions and grading
   * boxes stop at it. The adjoint accepts periodic contexts only. */
  int bc[4];
  /* Half-width gamma of the prediction stencil (Table 1): 1, 2 or 3 (0 reads
   * as 1), shared by the batch. It sets the grading box (+-gamma cells of the
   * parent level), the transport box (+-2 gamma cells of the leaf's level) and
   * the neighbours whose details correct it (+-gamma). gamma > 1 takes the
   * general transport path for every leaf (about five times the transport's
   * cost of gamma = 1). With a wall, 2^jmin >= 2 gamma. The adjoint accepts
   * gamma = 1 only. */
  int gamma;
  /* Sibling metric of the details (section "Mesh coarsening"):
   * MRLBM_METRIC_MAX, the max norm over the 2^d siblings, or MRLBM_METRIC_L2,
   * the l2 form 2^{-d/2} (sum of their squares)^{1/2} of the section's
   * footnote, which the library compares squared (2^{-d} times the sum of
   * squares against the squared thresholds). May differ per instance. */
  int metric;
  /* MRLBM_D3Q6: the advection velocity (V_x, V_y, V_z) of the equilibrium;
   * ignored by the other schemes. */
  double velocity[3];
} mrlbm_params;

#define MRLBM_METRIC_MAX 0
#define MRLBM_METRIC_L2 1

#define MRLBM_PERIODIC 0
#define MRLBM_COPY 1
#define MRLBM_BOUNCE_BACK 2
#define MRLBM_ANTI_BOUNCE_BACK 3

/* A context runs a batch of `batch` independent instances (1 <= batch <= 256),
 * p[0..batch-1], that share the scheme, the precision and jmin; jmax, eps,
 * mu_bar, lambda and the relaxation rates may differ per instance. Every step
 * advances all of them with one set of launches. Their total cell count
 * (sum over instances and levels of N_l^d) must stay below 2^31. */

/* Bytes of device workspace a context with these parameters needs.
 * Errors: MRLBM_ERR_INVALID for invalid parameters or a null pointer. */
int mrlbm_workspace_size(const mrlbm_params *p, int batch, size_t *bytes);

/* Create a context inside `workspace` (device memory, >= mrlbm_workspace_size
 * bytes, 256-byte aligned) that enqueues its work on `stream` (a hipStream_t,
 * NULL = the default stream). Uploads the parameter-dependent tables; does not
 * set an initial state. The launch schedule starts at its default (graph
 * replay, transport kernel chosen by problem size); mrlbm_set_tuning and
 * mrlbm_autotune change it. Reads no environment variable.
 * Errors: MRLBM_ERR_INVALID, MRLBM_ERR_CAPACITY, MRLBM_ERR_HIP. */
int mrlbm_create(const mrlbm_params *p, int batch, void *workspace, size_t ws_bytes, void *stream,
                 mrlbm_ctx **out);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same context as
 * mrlbm_create, with its workspace in a device array of the library itself,
 * MRLBM_STATIC_WORKSPACE_BYTES (16 MiB) on every GPU the library runs on, held
 * until the process ends. Enough for a D1Q2 or D1Q3 instance up to level 14 or
 * a D2Q9 instance up to level 8 in either precision; mrlbm_workspace_size tells
 * whether a configuration fits. The context runs on the current device; every
 * kernel of it uses that device's array, so at most one static context may be
 * alive per device at a time (a second create fails with MRLBM_ERR_STATE until
 * the first is destroyed; two contexts sharing the array would race). The array
 * keeps the last context's contents: creation clears what must start at zero,
 * as mrlbm_create does for a fresh workspace. Neither this call nor any later
 * call on the context allocates device memory: its steps launch the kernels
 * one by one (mrlbm_set_tuning with graph = 1 and mrlbm_autotune return
 * MRLBM_ERR_STATE), and everything else behaves as for mrlbm_create, with
 * identical results. The adjoint still takes the caller's adjoint workspace.
 * Errors: MRLBM_ERR_INVALID, MRLBM_ERR_CAPACITY (the workspace would exceed
 * MRLBM_STATIC_WORKSPACE_BYTES), MRLBM_ERR_STATE (a static context is alive on
 * this device), MRLBM_ERR_HIP. */
#define MRLBM_STATIC_WORKSPACE_BYTES (16u << 20)
int mrlbm_create_static(const mrlbm_params *p, int batch, void *stream, mrlbm_ctx **out);

/* Initial state of Algorithm 1 for one instance: the full finest mesh with
 * f = M^{-1} m_eq(m0) on every finest cell. `moments` is a device buffer in the
 * context precision, layout [nc][N_J^d] (see above). Every instance must be
 * initialised (or set) before the first step. Asynchronous. */
int mrlbm_init_equilibrium(mrlbm_ctx *ctx, int instance, const void *moments);

/* Mesh adaptation only: new tree G(H_eps(T_eps(tree))) with details of the
 * current leaf values, then the transfer of the data to the new complete leaves
 * (projection on merged cells, prediction on created ones). Asynchronous. */
int mrlbm_adapt(mrlbm_ctx *ctx);

/* Transport and collision on the current complete leaves, without adaptation
 * (the mesh is frozen for this call), after the reconstruction of the current
 * mesh. Right after mrlbm_adapt that reconstruction recomputes only the
 * projections above cells the adaptation changed (the others are still exact
 * in the context's buffers); otherwise, and after mrlbm_set_state or
 * mrlbm_init_equilibrium, all of them. Same results either way.
 * Asynchronous. */
int mrlbm_transport_collide(mrlbm_ctx *ctx);

/* `nsteps` full time steps of Algorithm 1 (adapt, transport, collide).
 * Asynchronous; nsteps >= 0. Each step is replayed from a HIP graph captured
 * on the context's first step in that buffer state (on a private stream, then
 * launched on the context stream); with mrlbm_tuning.graph = 0 the kernels are
 * launched one by one instead. Results are identical. */
int mrlbm_step(mrlbm_ctx *ctx, int nsteps);

/* One time step with the mesh adaptation replaced by given meshes (frozen /
 * replay mode, e.g. to repeat a recorded run's mesh sequence for finite
 * differences): `trees` (host) holds the membership bytes of the new complete
 * tree of every instance, concatenated in instance order, each in the tree
 * layout above. The step then transfers the leaf data to the new leaves
 * (section "Construction of the time adaptive mesh": copy, projection on
 * merged cells, prediction on created ones), transports and collides, as
 * mrlbm_step does after its adaptation. Each tree must be graded and complete
 * (as for mrlbm_set_state) and may refine the current tree by at most one
 * level (every new cell outside the current tree has its parent in it), as
 * an adaptation does. Synchronises the stream for the host checks, then
 * enqueues the step. Errors: MRLBM_ERR_INVALID (a tree fails the checks;
 * nothing is changed), MRLBM_ERR_STATE before initialisation. */
int mrlbm_step_frozen(mrlbm_ctx *ctx, const uint8_t *trees);

/* The current complete tree of one instance (membership bytes, tree layout
 * above) into a host buffer of mrlbm_sizes' total_cells bytes. Synchronous. */
int mrlbm_get_mesh(mrlbm_ctx *ctx, int instance, uint8_t *tree);

/* Copy the current tree and values of one instance to host buffers (layouts
 * above; `values` holds q * total_cells reals of the context precision): the
 * state of Algorithm 1 after the last collision. Only the complete leaves carry
 * the state; the other cells hold scratch (reconstruction values or stale data)
 * that depends only on the sequence of calls since mrlbm_create. Synchronous;
 * for device-side access to the leaves alone see mrlbm_fields. */
int mrlbm_get_state(mrlbm_ctx *ctx, int instance, uint8_t *tree, void *values);

/* Replace the current state by a host-side tree (must be a graded complete
 * tree: level jmin full, sibling groups complete, every tree cell's prediction
 * stencil in the tree, up to the walls) and leaf values. Synchronous.
 * Errors: MRLBM_ERR_INVALID if the tree is not graded and complete. */
int mrlbm_set_state(mrlbm_ctx *ctx, int instance, const uint8_t *tree, const void *values);

/* Total number of cells of one instance over levels jmin..jmax, and the number
 * of populations. */
int mrlbm_sizes(const mrlbm_ctx *ctx, int instance, int64_t *total_cells, int *q);

/* Diagnostics of one instance (synchronous): mass = sum over complete
 * leaves of |C_l| / |C_J| * sum_h f^h, the first conserved moment integrated
 * over the domain in units of finest cells (the quantity the adapted scheme
 * conserves: eq. (AdaptiveAdvectionPhase) telescopes over the leaves, which
 * partition the domain), accumulated in double with compensated (Neumaier)
 * summation in a fixed order, in either precision; per-level counts of
 * complete leaves (the set S(Lambda) of section "Tree structure and grading"; their sum
 * over levels divided by N_J^d is the mesh occupation rate of the numerical
 * experiments), internal tree cells and ghost cells ([jmax + 1] each, any of
 * them may be NULL).
 * Errors: MRLBM_ERR_NONFINITE if a leaf value of this instance is not finite
 * (the outputs are still written; the mass is then not finite); MRLBM_ERR_SYNC
 * (takes precedence) if the sticky wait flag is set. */
int mrlbm_stats(mrlbm_ctx *ctx, int instance, double *mass, int64_t *leaves, int64_t *internal,
                int64_t *ghosts);

/* Export of the complete leaves of one instance (the set S(Lambda) of section
 * "Tree structure and grading", which carries the solution of Algorithm 1) to device
 * buffers, in the order (level, cell):
 * `cells` receives (level << 26) | cell as uint32 and `values` receives q reals
 * per leaf ([leaf][h], context precision). `capacity` is the number of leaves
 * the buffers hold; *count receives the number of leaves. Synchronous.
 * Errors: MRLBM_ERR_CAPACITY if capacity < count (nothing is written). */
int mrlbm_leaves(mrlbm_ctx *ctx, int instance, uint32_t *cells, void *values, int64_t capacity,
                 int64_t *count);

/* Fields of one instance into a device buffer `out` of `out_bytes` bytes;
 * *n_written receives the number of elements (also when the buffer is too
 * small, so a first call with out = NULL, out_bytes = 0 sizes it):
 *   MRLBM_FIELD_LEAF_TABLE  uint32 [n]: (level << 26) | cell of every complete
 *                           leaf, in the order (level, cell);
 *   MRLBM_FIELD_POPULATIONS real [n][q]: the leaf populations, same order;
 *   MRLBM_FIELD_MOMENTS     real [n][q]: m = M f on every leaf, same order (M
 *                           of the scheme, section "Lattice Boltzmann schemes
 *                           on volumes"; D2Q9: the matrix of the Navier-Stokes
 *                           section, rows scaled by powers of lambda);
 *   MRLBM_FIELD_FINEST      real [q][N_J^d]: the reconstruction of every
 *                           population on the finest level (the double-hat
 *                           operator of section "Mesh coarsening": projection
 *                           up the tree, then zero-detail prediction down to J
 *                           on every cell outside it).
 * real is the context precision. MRLBM_FIELD_FINEST rewrites reconstruction
 * scratch of the context (never a leaf). Synchronous.
 * Errors: MRLBM_ERR_CAPACITY (nothing written), MRLBM_ERR_INVALID,
 * MRLBM_ERR_STATE before initialisation, MRLBM_ERR_SYNC. */
#define MRLBM_FIELD_LEAF_TABLE 1
#define MRLBM_FIELD_POPULATIONS 2
#define MRLBM_FIELD_MOMENTS 3
#define MRLBM_FIELD_FINEST 4
int mrlbm_fields(mrlbm_ctx *ctx, int instance, int what, void *out, size_t out_bytes, int64_t *n_written);

/* Counters of the work done since the last mrlbm_profile call (all instances).
 * With profiling on, graph-replayed steps (mrlbm_step) bracket the transport
 * kernel of every 8th step (profile mode 1) or of every step (mode 2), starting
 * with the first, with HIP events inside the step graph; eager steps (tuning graph = 0, mrlbm_adapt /
 * mrlbm_transport_collide) time every phase of every step. transport_ms / timed_launches is the average
 * duration of the kernel over the timed launches. */
typedef struct {
  uint64_t leaf_updates;       /* complete leaves transported and collided, summed over launches */
  uint64_t transport_launches; /* launches of the transport-collision kernel */
  double transport_ms;         /* HIP-event time of the transport-collision kernel alone (timed launches) */
  double reconstruct_ms;       /* HIP-event time of the reconstructions before transport (eager steps) */
  double adapt_ms;             /* HIP-event time of the mesh adaptation and transfer (eager steps) */
  uint64_t timed_launches;     /* transport launches covered by the event timings */
} mrlbm_counters;

/* Reset the counters and switch HIP-event timing off (enable = 0), on with
 * the transport kernel of every 8th graph-replayed step bracketed (1), or on
 * with that kernel of every graph-replayed step bracketed (2). Leaf updates are
 * always counted (on the device, by the transport kernel). Timing records
 * events on the context stream (see mrlbm_counters for which launches are
 * timed); each bracketing event costs the step a few microseconds.
 * Errors: MRLBM_ERR_INVALID for another value of enable. */
int mrlbm_profile(mrlbm_ctx *ctx, int enable);

/* Read the counters (synchronous). */
int mrlbm_read_counters(mrlbm_ctx *ctx, mrlbm_counters *out);

/* ---- Adjoint on frozen meshes (contexts with batch = 1) ----
 * The gradient of a functional J of the final leaf values with respect to the
 * initial conserved moments and the relaxation rates, for the run of Algorithm 1
 * whose meshes are held fixed (the adjoint of collision + MR transport +
 * transfer on each recorded mesh; no derivative through the thresholding).
 * Checkpoints every `ckpt_every` steps; each segment is recomputed forward with
 * a tape of its meshes and pre-collision populations, then swept backwards
 * (the workspace holds two such tapes: the recomputation of one segment runs
 * on the context stream while the previous one is swept on a second stream).
 * With ckpt_every >= nsteps (one segment) the recorded forward writes the tape
 * itself, the workspace holds one tape of nsteps steps, and the adjoint
 * recomputes nothing: the HBM-for-time trade when the tape fits.
 * Periodic boundaries, gamma = 1 and the schemes D1Q2, D1Q3 and D2Q9 only
 * (MRLBM_ERR_INVALID with a wall, gamma > 1 or the Euler scheme). */

/* Bytes of device workspace the adjoint of an `nsteps` run needs. */
int mrlbm_adjoint_workspace_size(const mrlbm_ctx *ctx, int nsteps, int ckpt_every, size_t *bytes);

/* Run `nsteps` steps from the current state (normally just after
 * mrlbm_init_equilibrium), storing checkpoints in `adj_workspace` (device,
 * caller-owned, kept until mrlbm_adjoint). Asynchronous.
 * Errors: MRLBM_ERR_CAPACITY if the workspace is too small. */
int mrlbm_forward_record(mrlbm_ctx *ctx, void *adj_workspace, size_t bytes, int nsteps, int ckpt_every);

/* Backward sweep of the recorded run (creates and destroys a stream of default
 * priority for the sweep). `abar_final` (device, values layout of the
 * final state; only complete-leaf entries are read) is dJ/d(final leaf values);
 * writes dJ/d(initial conserved moments) to `mbar0` (device, [nc][N_J^d], context
 * precision; meaningful when the run started from mrlbm_init_equilibrium) and
 * dJ/ds_k (k = 0..q-1, summed in double) to the host array `sbar`. Synchronous.
 * Leaves the context state unspecified (re-initialise or set it before stepping). */
int mrlbm_adjoint(mrlbm_ctx *ctx, const void *abar_final, void *mbar0, double *sbar);

/* ---- Launch schedule and its autotuner ----
 * The list kernels (projection, prediction, details, transfer, transport) run
 * a capped number of blocks that stride over the chunks of 64 list items; the
 * transport and the details have a per-item variant (one thread per leaf or
 * internal parent, all populations in it) and a per-population variant (one
 * wavefront per population), chosen together; the finest two links of the
 * level chains can share a launch (pair_links). The autotuner times
 * every schedule of a small grid on the context's current state (steps that
 * leave the state unchanged, replayed from HIP graphs between HIP events),
 * keeps the fastest, and caches it for the process per (device architecture,
 * scheme, precision, floor(log2(leaves)), walls present, gamma, sibling
 * metric). Schedules do not change results. */
typedef struct {
  int transport_variant; /* transport and details: 1 one thread per item, 2 one wavefront per population */
  int list_grid_all;     /* block cap of the all-level list kernels (8..65536) */
  int list_grid_level;   /* block cap of the per-level list kernels (8..65536) */
  int graph;             /* 1: steps replayed from HIP graphs (default); 0: kernels launched one by one */
  int pair_links;        /* 1: the two finest links of the projection, ghost and ancestor chains share a
                          * launch, the second half's blocks waiting on a device counter for the first
                          * half when both have work (one launch fewer; each waiting block then pays a
                          * device-scope release of the first half's blocks); 0 (default): one launch
                          * per link */
  int from_cache;        /* set by mrlbm_autotune: 1 if taken from the cache */
  double ms_per_step;    /* set by mrlbm_autotune: timed cost of the schedule (0 if cached) */
} mrlbm_tuning;

/* Time the candidate schedules with `reps` steps each and adopt the fastest.
 * Synchronous; the state and the leaf counters are unchanged. Needs graph
 * stepping (tuning graph = 1). Errors: MRLBM_ERR_STATE before initialisation
 * or without graph stepping. */
int mrlbm_autotune(mrlbm_ctx *ctx, int reps, mrlbm_tuning *chosen);
/* Adopt a schedule / read the current one. */
int mrlbm_set_tuning(mrlbm_ctx *ctx, const mrlbm_tuning *t);
int mrlbm_get_tuning(const mrlbm_ctx *ctx, mrlbm_tuning *out);

/* Plain device copy of `bytes` (a multiple of 16, both pointers 16-byte
 * aligned) on `stream`: the reference kernel for bandwidth and for the scale
 * of hardware traffic counters. Asynchronous. */
int mrlbm_copy(void *dst, const void *src, size_t bytes, void *stream);

/* Test hook of the paired launches' bounded wait: sets its spin budget
 * (0 = the default, about 50 ms) and overwrites the counter the waits poll
 * with `count`. A large negative count makes every ordered wait give up after
 * `budget` spins, so that the failure path (MRLBM_ERR_SYNC) can be exercised
 * while every kernel still runs to its end. For tests only: the context's
 * results are invalid afterwards. Synchronous. */
int mrlbm_debug_pair_wait(mrlbm_ctx *ctx, uint32_t budget, int32_t count);

/* Destroy the context (the workspace is the caller's to free). */
int mrlbm_destroy(mrlbm_ctx *ctx);

/* Human-readable text of a status code (static storage). */
const char *mrlbm_status_string(int status);

/* Host-side flattened transport weights of eq. (PredictionWithMatrixNew) for a
 * leaf n = jmax - l >= 1 levels above the finest, velocity h of `scheme`:
 *   W[h][25]: weight of the leaf-level value at offset (a, b) in [-2, 2]^2,
 *             index (b + 2) * 5 + (a + 2), of sum_E f^hat-hat - sum_A f^hat-hat
 *             (1D: the same layout, with only the row b = 0 nonzero);
 *   C[h][36]: weight of the detail of the level-(l+1) cell at offset (y1, y2)
 *             in [-2, 3]^2 from 2k, index (y2 + 2) * 6 + (y1 + 2) (1D: only
 *             the row y2 = 0 nonzero).
 * Pure host computation (no device, no context). Errors: MRLBM_ERR_INVALID,
 * also for MRLBM_D3Q6, which has no table of its own: its leaves apply the
 * D1Q2 rows of their velocity's sign along the velocity's axis (the sums of
 * the 3D reconstruction over a face collapse onto the leaf's row). */
int mrlbm_transport_tables(int scheme, int n, double *W, double *C);

/* The tables of the general transport path (walls, gamma > 1): as above for a
 * prediction of half-width gamma (1..3, Table 1), over the boxes of half-width
 * R = 2 gamma, for a leaf touching the walls named by wall_x, wall_y (0 none,
 * 1 the lower wall, 2 the upper one; 1D: wall_y = 0) of section "Boundary
 * conditions". The sums over E leave out the finest cells beyond the walls.
 *   W[h][(2R+1)^d]: offsets (a, b) in [-R, R]^d, index (b + R)(2R+1) + (a + R)
 *                   (1D: a + R);
 *   C[h][(2R+2)^d]: offsets (y1, y2) in [-R, R+1]^d from 2k, index
 *                   (y2 + R)(2R+2) + (y1 + R) (1D: y1 + R);
 *   N[h][2]:        the number of finest cells of E beyond the x wall and,
 *                   with x inside, beyond the y wall (their values come from the
 *                   wall's condition, eq. AdvectionOnBoundary).
 * Pure host computation. Errors: MRLBM_ERR_INVALID. */
int mrlbm_transport_tables_general(int scheme, int n, int gamma, int wall_x, int wall_y, double *W, double *C,
                                   double *N);

#ifdef __cplusplus
}
#endif
#endif
