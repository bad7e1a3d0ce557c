/*
 * pond.h -- C ABI of the MI355X particles-on-demand (PonD) f+g step library
 * (libpond.so).
 *
 * The library advances the double-distribution-function BGK model in its
 * total-energy split (Hosseini, Bhadauria, Karlin, arXiv:2405.11489, Sec. II,
 * Eq. total_energy_g and the first g-equation; the internal-energy split of
 * Eqs. int_energy_g, int_g_evolution on request) on the D2Q16 lattice of Table I,
 * with particle velocities shifted and scaled to each node's frame (u, T)
 * (Sec. "Discrete velocity solver ...: PonD"), semi-Lagrangian streaming with
 * Lagrange interpolation and the frame transformation of Sec. "Frame
 * transformation" (Eq. propagationInterpolated and Eqs. gradGeneralTransform,
 * a0..a3).  The destination frame of every node is found by a
 * predictor-corrector fixed-point iteration; converged populations are
 * re-projected onto the frame of their own moments and relaxed with BGK.
 *
 * Units are lattice units (dx = dt = 1, r = 1, rT_L = 1).  Fields are 2-D,
 * nx * ny nodes, row-major with x fastest (node n = y*nx + x).
 *
 * Conventions shared by every entry point:
 *   - Every function returns a pond_status unless stated otherwise; on error it
 *     leaves its outputs untouched and records a message readable through
 *     pond_last_error() (thread-local).
 *   - Field pointers (double) may be host memory or device memory of the
 *     context's GPU (e.g. torch tensor data pointers); the library detects which.
 *     The library only reads or writes them during the call (device pointers:
 *     in stream order on the context's stream) and never retains or frees them.
 *   - All work is enqueued on the context's HIP stream.  Calls that return
 *     data to the caller, pond_stats and pond_synchronize synchronise that
 *     stream; pond_step does not.
 *   - One host thread may use a given context at a time.
 *   - Device-side failure flags (density or temperature <= 0, non-finite
 *     values) surface as POND_ERR_NONPHYSICAL at the next synchronising call
 *     (stencils beyond a wall's ghost rows as POND_ERR_UNSUPPORTED); the
 *     context then refuses further steps with POND_ERR_STATE.
 */
#ifndef POND_H
#define POND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define POND_ABI_VERSION 3

/* Exported symbols (the library is built with hidden default visibility). */
#if defined(__GNUC__)
#define POND_API __attribute__((visibility("default")))
#else
#define POND_API
#endif

typedef struct pond_ctx pond_ctx; /* opaque; created by pond_create, owned by the library */

typedef enum {
    POND_OK = 0,
    POND_ERR_INVALID_ARG = 1,   /* a parameter or input field is out of range */
    POND_ERR_UNSUPPORTED = 2,   /* a valid option the library does not implement */
    POND_ERR_OUT_OF_MEMORY = 3, /* device allocation failed or caller memory too small */
    POND_ERR_DEVICE = 4,        /* a HIP runtime call or kernel launch failed */
    POND_ERR_NONPHYSICAL = 5,   /* the state produced rho <= 0, T <= 0 or NaN/Inf */
    POND_ERR_STATE = 6          /* call not valid in the context's current state */
} pond_status;

/* Lattice: Table I.  D2Q16 = D1Q4 x D1Q4, the fourth-order Gauss-Hermite rule
 * (abscissae +-sqrt(3 -+ sqrt 6), weights (3 +- sqrt 6)/12), Grad order 3.
 * D2Q25 = D1Q5 x D1Q5, the fifth-order rule (abscissae 0, +-sqrt(5 -+ sqrt 10),
 * weights 8/15, (7 +- 2 sqrt 10)/60), Grad order 4: the frame transformation
 * keeps the moments up to order four, which the non-translational split needs
 * for f (Sec. II).  D2Q25 runs the cubic stencil (interp_points = 3:
 * POND_ERR_UNSUPPORTED) with each of the three energy splits. */
enum { POND_LATTICE_D2Q16 = 16, POND_LATTICE_D2Q25 = 25 };

/* Energy split: Eqs. Es.
 *   POND_SPLIT_TOTAL: g carries the total energy (Eq. total_energy_g,
 *     g^eq = (U'/rho + v^2/2) f^eq) and has no source (the paper's choice).
 *   POND_SPLIT_INTERNAL: g carries the internal energy (Eq. int_energy_g,
 *     g^eq = (U'/rho + (v - u)^2/2) f^eq, sum g = rho c_v T) and, after the
 *     collision, receives the source of Eq. int_g_evolution once per step,
 *     S_i = -f_i (C_i - u) . (d_t u + C_i . grad u), with f the step's
 *     time-centred populations (the mean of the re-projected pre-collision and
 *     the collided f, whose stress is the physical one), d_t u the new minus
 *     the old frame velocity of the node and grad u central differences of the
 *     neighbours' old frame velocities (the boundary rule of bc_x / bc_y picks
 *     the neighbours; beyond a wall, the ghost frame velocity).
 *     With prandtl != 1, g relaxes at 1/tau_1 (its flux is the heat flux).
 *   POND_SPLIT_NONTRANS: g carries the non-translational energy (Eq. nt_energy_g,
 *     g^eq = (U'/rho) f^eq, U' = rho (c_v - 1) T); the energy is
 *     E = sum (g + |C_i|^2 f / 2).  Built with the paper's BGK only: prandtl
 *     must be 1 (else POND_ERR_UNSUPPORTED). */
enum { POND_SPLIT_TOTAL = 0, POND_SPLIT_INTERNAL = 1, POND_SPLIT_NONTRANS = 2 };

/* Arithmetic of the step.  FP64: everything in double.  FP32: populations,
 * interpolation and frame transformation in float; conserved-moment sums,
 * temperature recovery and the predictor-corrector test in double. */
enum { POND_PREC_FP64 = 0, POND_PREC_FP32 = 1 };

/* Boundary handling per axis: periodic wrap, or clamp (zero-gradient: a
 * stencil index beyond the edge is replaced by the edge node, populations and
 * frame alike), or (bc_y only) walls, for the thermal Couette flow of Sec.
 * "Measuring viscous heating" (the paper gives no boundary scheme; this one is
 * a reading).  Walls at y = -1/2 (bottom) and y = ny - 1/2 (top) move along x
 * at wall_ux[0 | 1] and are held at wall_T[0 | 1].  A stencil row beyond a wall
 * is a ghost mirroring the interior row at the same distance: its velocity and
 * temperature continue the mirror node's linearly through the wall
 * (u_g = 2 U_w - u_m with the normal component reversed, T_g = 2 T_w - T_m, at
 * least T_w / 4), its density keeps the mirror's pressure, and its moments are
 * the equilibrium moments of that state plus the mirror's non-equilibrium
 * moments.  The ghost rows reach 8 rows beyond each wall: every departure
 * stencil must stay within them, i.e. near the bottom wall, for a node on row
 * y, floor(y - c_out sqrt(T) - u_y) - 1 >= -8 with the cubic stencil (at
 * rest on the first row: c_out sqrt(T) <= 7, T <= 8.99 on D2Q16, 6.00 on
 * D2Q25; c_out = 2.33 on D2Q16, 2.86 on D2Q25), likewise at the top wall.
 * A frame that reaches further is refused at pond_init_fields and
 * pond_import_state (POND_ERR_UNSUPPORTED); an iterate frame that gets there
 * during a step is flagged on the device and reported as
 * POND_ERR_UNSUPPORTED at the next synchronising call, after which the
 * context is in the error state (as for POND_ERR_NONPHYSICAL).  Walls run
 * every split on both lattices, in batches and the server too. */
enum { POND_BC_PERIODIC = 0, POND_BC_CLAMP = 1, POND_BC_WALL = 2 };

typedef struct {
    uint32_t struct_size;  /* = sizeof(pond_params); ABI guard */
    int32_t nx, ny;        /* nodes per axis, >= 1, nx * ny <= 2^31 - 1; ny == 1 is a
                              quasi-1-D run */
    int32_t bc_x, bc_y;    /* POND_BC_*; POND_BC_WALL for bc_y only */
    int32_t lattice;       /* POND_LATTICE_D2Q16 (default) or POND_LATTICE_D2Q25 */
    int32_t interp_points; /* 4 = cubic Lagrange (default); 3 = quadratic, the paper's
                              "2nd-order" stencil (end of Sec. "Streaming") */
    int32_t split;         /* POND_SPLIT_TOTAL (default), POND_SPLIT_INTERNAL or
                              POND_SPLIT_NONTRANS */
    int32_t precision;     /* POND_PREC_* */
    int32_t pc_max_iter;   /* predictor-corrector cap; <= 0 selects 32 */
    double tau;            /* relaxation time in lattice units, > 1/2; the discrete
                              step has kinematic viscosity nu = (tau - 1/2) T
                              (Eq. kin_visc with the dt/2 shift of the discrete BGK) */
    double prandtl;        /* > 0.  1 = the paper's single-relaxation-time BGK
                              (Pr = 1, Sec. II); otherwise the Fourier part of the
                              energy flux relaxes with tau_1 = 1/2 + (tau - 1/2)/Pr
                              (quasi-equilibrium extension referred to in Sec. II) */
    double gamma;          /* adiabatic exponent, 1 < gamma <= 2 (Eq. spec_heat,
                              c_v = 1/(gamma - 1) >= D/2 keeps U' >= 0) */
    double pc_tol;         /* predictor-corrector tolerance on
                              max(|du|_inf / sqrt(T), |dT| / T_E); <= 0 selects 1e-13
                              (FP64) or 1e-6 (FP32).  T_E = T in FP64; in FP32
                              T_E = E / (rho c_v), the scale of the energy T is
                              recovered from (T + |u|^2 / (2 c_v) in the total split,
                              T in the internal split) */
    double wall_ux[2];     /* bc_y = POND_BC_WALL: x-velocity of the bottom / top wall */
    double wall_T[2];      /* bc_y = POND_BC_WALL: temperature of the bottom / top wall, > 0 */
} pond_params;

/* Per-context counters since the last pond_init_fields / pond_import_state. */
typedef struct {
    int64_t steps;            /* steps completed */
    int64_t node_updates;     /* steps * nodes */
    int64_t pc_iterations;    /* predictor-corrector gathers summed over nodes and steps */
    int64_t nonconverged;     /* node-steps that stopped at pc_max_iter (not an error) */
    int32_t nonphysical;      /* non-zero once a non-physical node was produced */
    int32_t reserved;
} pond_stats_t;

/* ABI version of the loaded library (POND_ABI_VERSION). */
POND_API int pond_abi_version(void);

/* Fill *p with defaults: D2Q16, total split, cubic stencil, FP32, periodic,
 * tau = 0.6, Pr = 1, gamma = 1.4, default tolerance and cap; nx = ny = 0 (the
 * caller must set the size). */
POND_API pond_status pond_params_default(pond_params *p);

/* Bytes of device memory a context with these parameters uses (two state
 * buffers, two sets of moment planes, counters), or 0 if *p is invalid.
 * D2Q16: FP32 464 B per node (2 x 152 B of state, 2 x 80 B of moments), FP64
 * 880 B (2 x 280 + 2 x 160); D2Q25: FP32 704 B, FP64 1328 B; the
 * internal-energy split adds 2 x 16 B (each buffer keeps the previous level's
 * frame velocities); walls add the moment planes' ghost rows (16 rows); plus a
 * few KiB. */
POND_API size_t pond_state_bytes(const pond_params *p);

/* Create a context.  Validates *p before touching the device: invalid values
 * give POND_ERR_INVALID_ARG, valid but unimplemented options
 * POND_ERR_UNSUPPORTED, and *out is left NULL.
 *   hip_stream:  hipStream_t to enqueue work on; NULL = a stream the context
 *                creates (default priority) and destroys.
 *   device_mem:  NULL = the library allocates pond_state_bytes(p) with
 *                hipMalloc and frees it in pond_destroy; otherwise caller-owned
 *                device memory of at least device_mem_bytes >= pond_state_bytes(p)
 *                bytes, 256-byte aligned, which the library never frees.
 * The state is undefined until pond_init_fields or pond_import_state. */
POND_API pond_status pond_create(const pond_params *p, void *hip_stream, void *device_mem,
                        size_t device_mem_bytes, pond_ctx **out);

/* Initialise every node at equilibrium in its own frame: f_i = rho w_i,
 * g_i = w_i [rho (c_v - 1) T + rho |C_i|^2 / 2] with C_i = sqrt(T) c_i + u
 * (Sec. "Discrete velocity solver ...: PonD" and the total-split g^eq of Sec.
 * II; the internal split puts C_i - u = sqrt(T) c_i in place of C_i), frame
 * (u, T).  Arrays of nx*ny doubles.  rho <= 0, T <= 0 or a
 * non-finite value anywhere gives POND_ERR_INVALID_ARG (the context is then
 * left uninitialised).  Synchronises the stream.  Resets the counters. */
POND_API pond_status pond_init_fields(pond_ctx *c, const double *rho, const double *ux, const double *uy,
                             const double *T);

/* Advance nsteps >= 0 steps, asynchronously on the context stream.  One step
 * updates every node (Jacobi: each reads only the state of the previous step):
 * the populations of each velocity are gathered at its departure point
 * x - C_i dt by Lagrange interpolation over the stencil nodes, each stencil
 * node's populations taken from its own frame into the node's frame (Sec.
 * "Frame transformation", Eqs. gradGeneralTransform, a0..a3, Eq.
 * propagationInterpolated), the node's frame is found by the
 * predictor-corrector iteration on the gathered moments, and f and g relax
 * toward their equilibria (Sec. II, the BGK equations of f and g).  Refused
 * (POND_ERR_STATE) before initialisation, while the context is a batch member
 * or once it is in the error state. */
POND_API pond_status pond_step(pond_ctx *c, int64_t nsteps);

/* Macroscopic fields of the current state (Sec. II): rho = sum f, rho u =
 * sum f C_i, E = sum g, T = (E - rho |u|^2 / 2) / (rho c_v), p = rho T
 * (internal split: U = sum g, T = U / (rho c_v)).
 * Any output pointer may be NULL to skip it.  Synchronises the stream. */
POND_API pond_status pond_moments(pond_ctx *c, double *rho, double *ux, double *uy, double *T, double *p);

/* Copy the counters; synchronises the stream. */
POND_API pond_status pond_stats(pond_ctx *c, pond_stats_t *out);

/* Wait for the context's stream and report device-side flags. */
POND_API pond_status pond_synchronize(pond_ctx *c);

/* Raw state, converted to double: f and g as Q planes of nx*ny values (Q = the
 * lattice, 16 or 25; plane i = velocity i = q1 a + b with c_i = (c_a, c_b),
 * q1 = 4 or 5, c_a ascending), frame
 * as 3 planes (u_x, u_y, T), and the 2-vector reference velocity the FP32
 * moments are taken about (nullable; host memory).  Synchronises the stream. */
POND_API pond_status pond_export_state(pond_ctx *c, double *f, double *g, double *frame, double *u_ref);

/* Load a raw state in the layout of pond_export_state (FP32 contexts round to
 * float).  u_ref (host memory) may be NULL (mass-weighted mean velocity).
 * With walls, a frame whose departure stencils leave the ghost rows is
 * refused (POND_ERR_UNSUPPORTED).  Resets the counters.  Synchronises the
 * stream. */
POND_API pond_status pond_import_state(pond_ctx *c, const double *f, const double *g, const double *frame,
                              const double *u_ref);

/* The internal-energy split's previous time level: the frame velocities u_x,
 * u_y of the state before the current one, which the split's source uses (its
 * velocity gradient is extrapolated along each node's trajectory from the last
 * two levels, a reading of Eq. int_g_evolution, which gives the source's
 * gradient but no discretisation).  prev: 2 planes of nx*ny doubles (u_x, then
 * u_y), host or device memory.  After pond_init_fields or pond_import_state
 * the current frames stand in for the previous level; pond_import_prev_frame
 * (after pond_import_state) loads it, so an exported state resumes bit for bit.
 * Both synchronise the stream; other splits keep no previous level
 * (POND_ERR_UNSUPPORTED).  The import is refused while the context is a batch
 * member (POND_ERR_STATE); its values are taken as given. */
POND_API pond_status pond_export_prev_frame(pond_ctx *c, double *prev);
POND_API pond_status pond_import_prev_frame(pond_ctx *c, const double *prev);

/* Launch configuration of the step kernel (performance only: every
 * configuration computes the same numbers, bit for bit).
 *   kernel:    POND_KERNEL_TILED (default) stages each block's source region in
 *              LDS; POND_KERNEL_GLOBAL reads every tap from HBM (reference).
 *   tile:      POND_TILE_* block shape of the tiled kernel (destination nodes).
 *   lds_nodes: LDS capacity per block, in nodes (the 20 moments of a node,
 *              30 on D2Q25: D2Q16 80 B in FP32, 160 B in FP64; D2Q25 128 B
 *              in FP32 (30 floats and two of padding), 240 B in FP64); taps
 *              outside the staged region read HBM.  At most 159 KiB: one KiB of the CU's 160 stays for
 *              the kernels' static shared memory.
 *   batch_tile_width: tile of this context when it steps inside a pond_batch.
 * pond_set_tuning validates the values (POND_ERR_INVALID_ARG otherwise);
 * lds_nodes <= 0 selects the default for the tile.  Refused (POND_ERR_STATE)
 * while the context is a member of a batch. */
enum { POND_KERNEL_TILED = 0, POND_KERNEL_GLOBAL = 1 };
enum { POND_TILE_16x16 = 0, POND_TILE_32x8 = 1, POND_TILE_16x8 = 2, POND_TILE_8x8 = 3,
       POND_TILE_256x1 = 4, POND_TILE_64x1 = 5,
       POND_TILE_32x16 = 6 /* 512 lanes, D2Q16 only (POND_ERR_UNSUPPORTED on D2Q25) */ };
typedef struct {
    int32_t kernel;
    int32_t tile;
    int32_t lds_nodes;
    int32_t batch_tile_width;  /* batched step: tile width in {16, 32, 64, 128, 256}
                                  (height 256 / width); 0 = autotuned or default */
} pond_tuning;

POND_API pond_status pond_get_tuning(pond_ctx *c, pond_tuning *out);
POND_API pond_status pond_set_tuning(pond_ctx *c, const pond_tuning *t);

/* Kernel timing on the context stream, for measurement.  While enabled,
 * pond_step brackets each of its launches with HIP events; the results give
 * the summed device time of the moment pre-pass and of the step kernel over
 * the launches since profiling was enabled.  The step kernel writes the
 * moments of the state it produces, so the pre-pass runs only on the first
 * step after pond_init_fields or pond_import_state. */
typedef struct {
    int64_t launches;       /* steps timed */
    double prepass_ms;      /* summed duration of the moment pre-pass launches */
    double step_ms;         /* summed duration of the step-kernel launches (with the
                               wall ghost rows when bc_y is POND_BC_WALL) */
} pond_profile_t;

/* enable != 0 starts (and clears) timing; 0 stops it and drops pending events. */
POND_API pond_status pond_profile_enable(pond_ctx *c, int enable);

/* Synchronise, then report the timing accumulated since pond_profile_enable(c, 1). */
POND_API pond_status pond_profile_read(pond_ctx *c, pond_profile_t *out);

/* Release the context and the memory it allocated.  NULL-safe.  Refused
 * (POND_ERR_STATE) while the context is a member of a batch. */
POND_API pond_status pond_destroy(pond_ctx *c);

/* ------------------------------------------------- no-allocation step ----
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, serving loops that must not call hipMalloc.  The steps of
 * pond_step, on two state buffers the caller owns, with no context: the call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 *
 * The library's working memory for the steps (the moment planes of the two
 * states and the counters) is a fixed 64 MiB device workspace, one per GPU,
 * held until the process ends.  It holds grids of up to about 419 000 nodes
 * in FP32 on D2Q16 (e.g. 640 x 640), 209 000 in FP64 (456 x 456), 262 000 in
 * FP32 on D2Q25 (512 x 512); larger grids are refused with
 * POND_ERR_OUT_OF_MEMORY before any device work.  Every call on a GPU shares
 * that GPU's workspace and keeps nothing in it between calls (each call
 * clears its counters and recomputes the moments of its input): calls that
 * overlap on one GPU (other streams, other threads) race and must not be made.
 *
 * p:       the parameters of pond_create (validated the same way).
 * u_ref:   host pointer to the 2-vector reference velocity the FP32 moments
 *          are taken about (pond_export_state returns a context's), or NULL
 *          for (0, 0).  Results equal pond_step's bit for bit when it equals
 *          the context's.
 * f_a, g_a, frame_a: buffer A, the input state, device memory of the current
 *          GPU: Q planes of f, Q planes of g (float in FP32, double in FP64,
 *          plane i = velocity i, nx*ny values each, the layout of
 *          pond_export_state), and 3 planes u_x, u_y, T (double); with the
 *          internal-energy split 5 planes: u_x, u_y, T and the previous time
 *          level's u_x, u_y (pond_export_prev_frame).
 * f_b, g_b, frame_b: buffer B, the same layout, device memory.
 * nsteps:  >= 0 steps; A and B are ping-pong buffers: step k reads A and
 *          writes B when k is even, reads B and writes A when k is odd, so the
 *          result is in B when nsteps is odd and in A (overwritten) when it is
 *          even (nsteps = 0 leaves both untouched).
 * hip_stream: the stream to enqueue on (NULL: the null stream).  Asynchronous
 *          unless stats is given.
 * stats:   NULL, or host memory for the counters of these steps; then the call
 *          synchronises the stream (so it cannot be captured) and returns
 *          POND_ERR_NONPHYSICAL or POND_ERR_UNSUPPORTED (a wall's ghost rows
 *          overrun) as pond_stats would.
 * Errors: POND_ERR_INVALID_ARG (parameters, NULL or host buffers, nsteps < 0),
 * POND_ERR_UNSUPPORTED (options pond_create refuses), POND_ERR_OUT_OF_MEMORY
 * (grid larger than the workspace), POND_ERR_DEVICE (launch failure). */
POND_API pond_status pond_step_noalloc(const pond_params *p, const double *u_ref, void *f_a,
                                       void *g_a, double *frame_a, void *f_b, void *g_b,
                                       double *frame_b, int64_t nsteps, void *hip_stream,
                                       pond_stats_t *stats);

/* ------------------------------------------------------------- batches ----
 * A batch advances several contexts together, each by the same step as
 * pond_step (the step of Sec. "Discrete velocity solver ...: PonD" with
 * Eq. propagationInterpolated; results are bit for bit those of pond_step on
 * the member alone).  One batched step is one step launch over the tiles of
 * every member (one block per tile, each XCD taking a contiguous range of the
 * tile list), which also writes the moments of the state it produces; a
 * moment pre-pass over every member's nodes runs before it only when some
 * member's moments are stale (after pond_init_fields or pond_import_state).
 * Both launches are replayed from HIP graphs captured at creation.
 *
 * Members must be D2Q16 contexts (POND_ERR_UNSUPPORTED otherwise; walls
 * included: their ghost rows are refilled after every batched step),
 * initialised, not in the error state, not in another batch, and
 * share precision, interp_points and the energy split; sizes, boundary
 * conditions and physical parameters may differ.  While a context is a member it refuses
 * pond_step, pond_init_fields, pond_import_state, pond_set_tuning and
 * pond_destroy (POND_ERR_STATE); pond_moments, pond_stats and
 * pond_export_state stay available and see every batched step enqueued
 * before them.  The batch does not own its members: destroy the batch, then
 * the contexts. */
typedef struct pond_batch pond_batch; /* opaque */

typedef struct {
    int32_t members;      /* contexts in the batch */
    int32_t tiles;        /* tiles per batched step, all members */
    int32_t grid_blocks;  /* blocks of the step launch (one per tile; a build with
                             POND_BATCH_PERSISTENT=1 launches a fixed grid) */
    int32_t lds_nodes;    /* LDS capacity per block, in nodes */
    int64_t nodes;        /* nodes per batched step, all members */
    int64_t steps;        /* batched steps enqueued since creation */
    int32_t graph_steps;  /* steps per launch of the larger captured graph */
    int32_t reserved;
} pond_batch_info_t;

/* Build a batch of n contexts (array of n distinct handles, copied), which
 * share precision, interp_points, energy split and lattice (D2Q16 or D2Q25;
 * otherwise POND_ERR_INVALID_ARG).
 * hip_stream: stream of the batched steps (NULL: the batch creates its own).
 * Synchronises the members' streams.  Each member steps with tiles of width
 * pond_tuning.batch_tile_width, else the autotuned width of its size class,
 * else a default (32 in FP32, 16 in FP64, 256 for grids of fewer than 8
 * rows).  Allocates a small device table (members x ~200 bytes). */
POND_API pond_status pond_batch_create(pond_ctx *const *ctxs, int n, void *hip_stream,
                                       pond_batch **out);

/* Enqueue nsteps (>= 0) batched steps; asynchronous.  Refused
 * (POND_ERR_STATE) once a member is known to be in the error state. */
POND_API pond_status pond_batch_step(pond_batch *b, int64_t nsteps);

/* Wait for the batch's stream, then read every member's flags: members with
 * non-physical values enter the error state and the call returns
 * POND_ERR_NONPHYSICAL (the other members are unaffected and their results
 * stay valid). */
POND_API pond_status pond_batch_synchronize(pond_batch *b);

POND_API pond_status pond_batch_get_info(pond_batch *b, pond_batch_info_t *out);

/* Tile width the batch uses for member i (0 <= i < members). */
POND_API pond_status pond_batch_member_tile_width(pond_batch *b, int i, int *width);

/* Synchronise, release the batch's graphs and table, and return the members
 * to single-context use.  NULL-safe. */
POND_API pond_status pond_batch_destroy(pond_batch *b);

/* Autotuner: time at least `steps` (>= 1) steps and 2 ms of device time of c
 * with each candidate tile shape and LDS capacity of the single-context
 * kernel and each candidate batch tile width (one-member batches), in two
 * interleaved rounds, restoring c's state, step count and counters after
 * every candidate.  A candidate replaces the default only when more than 3 %
 * faster.  Applies the result to c, stores it for c's class (lattice,
 * energy split, precision, stencil, boundary conditions, rounded log2 of nx
 * and of ny, and the stencil reach max(|u_x|, |u_y|) + c_out sqrt(T) of the
 * initial frame, rounded up)
 * in a process-wide cache that pond_init_fields / pond_import_state (unless
 * the tuning was set explicitly) and pond_batch_create consult, and returns
 * it in *out (nullable).  Allocates one state buffer's worth of device memory
 * while it runs.  Every candidate computes the same numbers. */
POND_API pond_status pond_autotune(pond_ctx *c, int steps, pond_tuning *out);

/* Forget every autotuned size class. */
POND_API pond_status pond_tuning_cache_clear(void);

/* -------------------------------------------------------------- serving ----
 * A server takes requests (parameters, initial fields, step count), queues
 * them first in, first out, and serves them with continuous batching: a worker
 * thread admits the head of the queue whenever its footprint
 * (pond_state_bytes) fits the HBM budget next to the admitted requests; each
 * round it steps, through one pond_batch (rebuilt when the selection
 * changes), the admitted requests with the least remaining work until the
 * round holds fill_nodes nodes (shortest-remaining-work first, filled to keep
 * the chip busy; a round's requests share the lattice -- and, in a server
 * configured with POND_SERVE_ANY, the precision, stencil or split -- of its
 * first one, so requests of different kinds take turns); it re-examines the queue every
 * chunk_steps steps and as soon as a request finishes, and releases a finished request's device memory
 * after copying its outputs to host memory.  Each request's results are those
 * of pond_step on it alone (the step of Sec. "Discrete velocity solver ...:
 * PonD"), whatever traffic it shared the GPU with.  All API calls are
 * thread-safe; the server owns every context it creates. */
typedef struct pond_server pond_server; /* opaque */

/* POND_SERVE_ANY in a server configuration's precision, interp_points or
 * split: the server takes requests of any value of that field, and a round
 * batches requests that agree on it (as on the lattice). */
enum { POND_SERVE_ANY = -1 };

typedef struct {
    uint32_t struct_size;      /* = sizeof(pond_server_config) */
    int32_t precision;         /* POND_PREC_* shared by all requests, or POND_SERVE_ANY
                                  (default FP32) */
    int32_t interp_points;     /* 3 or 4, shared by all requests, or POND_SERVE_ANY
                                  (default 4) */
    int32_t max_members;       /* cap on running requests; <= 0: none (default) */
    int64_t hbm_budget_bytes;  /* admission cap on the summed pond_state_bytes of running
                                  requests (default 64 GiB).  Transient buffers come on
                                  top of it: one request at a time, the staging of its
                                  initial fields (4 N doubles, inside its own state
                                  memory), the state copy of autotune_steps (one state
                                  buffer) and the export buffer of
                                  POND_REQ_KEEP_STATE ((2Q + 3) N doubles), each freed before
                                  the next request is admitted or collected */
    int64_t chunk_steps;       /* batched steps between queue checks; 0: run until the
                                  next request finishes (default 64) */
    int64_t fill_nodes;        /* each round steps the requests with the least remaining
                                  work (nodes x steps) until the round holds this many
                                  nodes; <= 0: every admitted request (of the round's
                                  kind; default 2^19) */
    int64_t autotune_steps;    /* > 0: pond_autotune (with this many steps) the first
                                  request of every new size class at admission
                                  (default 0) */
    int32_t split;             /* POND_SPLIT_* shared by all requests, or POND_SERVE_ANY
                                  (default TOTAL) */
} pond_server_config;

enum { POND_REQ_QUEUED = 0, POND_REQ_RUNNING = 1, POND_REQ_DONE = 2, POND_REQ_FAILED = 3 };
/* Request flags: outputs kept in host memory at completion. */
enum { POND_REQ_KEEP_MOMENTS = 1, /* rho, u_x, u_y, T, p: 5 N doubles */
       POND_REQ_KEEP_STATE = 2 }; /* pond_export_state layout + u_ref: (2Q + 3) N + 2
                                     doubles, Q = 16 on D2Q16 (35 N + 2), 25 on D2Q25
                                     (an internal-split server keeps no previous level:
                                     imported again, the state resumes as after
                                     pond_import_state alone) */

typedef struct {
    int32_t state;        /* POND_REQ_* */
    int32_t error;        /* pond_status of a failed request (POND_ERR_NONPHYSICAL, ...) */
    int64_t steps_done;
    int64_t steps_total;
    int64_t state_bytes;  /* its footprint against the budget */
    double t_submit;      /* seconds since pond_server_create (steady clock) */
    double t_admit;       /* -1 until admitted */
    double t_done;        /* -1 until finished; latency = t_done - t_submit */
} pond_request_info;

typedef struct {
    int64_t submitted, admitted, completed, failed;
    int64_t admission_waits;  /* rounds in which the queue head did not fit */
    int64_t batch_builds;     /* batches built (membership changes) */
    int64_t batched_steps;    /* batched steps run */
    int64_t node_updates;     /* node updates of all requests */
    int64_t queued, running;  /* now */
    int64_t used_bytes;       /* footprint of the running requests now */
    int64_t rounds;           /* batched rounds run */
    int64_t ns_admit;         /* worker time creating and initialising contexts */
    int64_t ns_build;         /* worker time building batches */
    int64_t ns_step;          /* worker time enqueueing and waiting for batched steps */
    int64_t ns_retire;        /* worker time collecting outputs and freeing contexts */
} pond_server_stats_t;

POND_API pond_status pond_server_config_default(pond_server_config *c);

/* Start a server (and its worker thread) on the current device, with its own
 * stream. */
POND_API pond_status pond_server_create(const pond_server_config *cfg, pond_server **out);

/* Queue a request.  The four fields (host memory, nx * ny doubles each, layout
 * of pond_init_fields) are copied before the call returns.  Requests whose
 * parameters are invalid, whose precision, interp_points or split differ from
 * the server's (unless it takes any), or whose footprint exceeds the whole budget are refused
 * (POND_ERR_INVALID_ARG); invalid field values fail the request at admission.
 * *id > 0 identifies it. */
POND_API pond_status pond_server_submit(pond_server *s, const pond_params *p, const double *rho,
                                        const double *ux, const double *uy, const double *T,
                                        int64_t nsteps, int32_t flags, int64_t *id);

POND_API pond_status pond_server_poll(pond_server *s, int64_t id, pond_request_info *out);

/* Block until request id has finished (id = 0: until every submitted request
 * has finished). */
POND_API pond_status pond_server_wait(pond_server *s, int64_t id);

/* Copy a finished request's kept outputs (nullable destinations; host
 * memory): moments 5 N doubles (rho, u_x, u_y, T, p), state (2Q + 3) N + 2
 * doubles (f, g, frame, u_ref as pond_export_state; Q = 16 on D2Q16, 25 on
 * D2Q25).  A failed request returns its
 * error. */
POND_API pond_status pond_server_result(pond_server *s, int64_t id, double *moments, double *state);

/* Drop a finished request's record and outputs. */
POND_API pond_status pond_server_release(pond_server *s, int64_t id);

POND_API pond_status pond_server_get_stats(pond_server *s, pond_server_stats_t *out);

/* Drop the queued requests, let the running ones finish, stop the worker and
 * free everything.  NULL-safe. */
POND_API pond_status pond_server_destroy(pond_server *s);

/* Static description of a status code (never NULL). */
POND_API const char *pond_status_string(pond_status s);

/* Message of the last error on the calling thread ("" if none). */
POND_API const char *pond_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* POND_H */
