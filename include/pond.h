/*
 * pond.h -- C ABI of the MI355X particles-on-demand (PonD) f+g step library
 * (libpond.so), ABI version 1.
 *
 * The library advances the double-distribution-function BGK model in its
 * total-energy split (Hosseini, Bhadauria, Karlin, arXiv:2405.11489, Sec. II,
 * Eq. total_energy_g and the first g-equation) on the D2Q16 lattice of Table I,
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
 *     values) surface as POND_ERR_NONPHYSICAL at the next synchronising call;
 *     the context then refuses further steps with POND_ERR_STATE.
 */
#ifndef POND_H
#define POND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define POND_ABI_VERSION 1

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
    POND_ERR_UNSUPPORTED = 2,   /* a valid option this build does not implement */
    POND_ERR_OUT_OF_MEMORY = 3, /* device allocation failed or caller memory too small */
    POND_ERR_DEVICE = 4,        /* a HIP runtime call or kernel launch failed */
    POND_ERR_NONPHYSICAL = 5,   /* the state produced rho <= 0, T <= 0 or NaN/Inf */
    POND_ERR_STATE = 6          /* call not valid in the context's current state */
} pond_status;

/* Lattice: Table I.  D2Q16 = D1Q4 x D1Q4, the fourth-order Gauss-Hermite rule
 * (abscissae +-sqrt(3 -+ sqrt 6), weights (3 +- sqrt 6)/12). */
enum { POND_LATTICE_D2Q16 = 16 };

/* Energy split: Eqs. Es.  Only the total-energy split (Eq. total_energy_g,
 * g^eq = (U'/rho + v^2/2) f^eq) is implemented; the others return
 * POND_ERR_UNSUPPORTED. */
enum { POND_SPLIT_TOTAL = 0, POND_SPLIT_INTERNAL = 1, POND_SPLIT_NONTRANS = 2 };

/* Arithmetic of the step.  FP64: everything in double.  FP32: populations,
 * interpolation and frame transformation in float; conserved-moment sums,
 * temperature recovery and the predictor-corrector test in double. */
enum { POND_PREC_FP64 = 0, POND_PREC_FP32 = 1 };

/* Boundary handling per axis: periodic wrap, or clamp (zero-gradient: a
 * stencil index beyond the edge is replaced by the edge node, populations and
 * frame alike). */
enum { POND_BC_PERIODIC = 0, POND_BC_CLAMP = 1 };

typedef struct {
    uint32_t struct_size;  /* = sizeof(pond_params); ABI guard */
    int32_t nx, ny;        /* nodes per axis, >= 1; ny == 1 is a quasi-1-D run */
    int32_t bc_x, bc_y;    /* POND_BC_* */
    int32_t lattice;       /* POND_LATTICE_D2Q16 */
    int32_t interp_points; /* 4 = cubic Lagrange (default); 3 = quadratic, the paper's
                              "2nd-order" stencil (end of Sec. "Streaming") */
    int32_t split;         /* POND_SPLIT_TOTAL */
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
                              max(|du|_inf / sqrt(T), |dT| / T); <= 0 selects 1e-13
                              (FP64) or 1e-6 (FP32) */
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
 * buffers, the moment planes and counters), or 0 if *p is invalid.  FP32:
 * 384 B per node; FP64: 720 B per node; plus a few KiB. */
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
 * II), frame (u, T).  Arrays of nx*ny doubles.  rho <= 0, T <= 0 or a
 * non-finite value anywhere gives POND_ERR_INVALID_ARG (the context is then
 * left uninitialised).  Synchronises the stream.  Resets the counters. */
POND_API pond_status pond_init_fields(pond_ctx *c, const double *rho, const double *ux, const double *uy,
                             const double *T);

/* Advance nsteps >= 0 steps, asynchronously on the context stream. */
POND_API pond_status pond_step(pond_ctx *c, int64_t nsteps);

/* Macroscopic fields of the current state (Sec. II): rho = sum f, rho u =
 * sum f C_i, E = sum g, T = (E - rho |u|^2 / 2) / (rho c_v), p = rho T.
 * Any output pointer may be NULL to skip it.  Synchronises the stream. */
POND_API pond_status pond_moments(pond_ctx *c, double *rho, double *ux, double *uy, double *T, double *p);

/* Copy the counters; synchronises the stream. */
POND_API pond_status pond_stats(pond_ctx *c, pond_stats_t *out);

/* Wait for the context's stream and report device-side flags. */
POND_API pond_status pond_synchronize(pond_ctx *c);

/* Raw state, converted to double: f and g as 16 planes of nx*ny values
 * (plane i = velocity i = 4a + b with c_i = (c_a, c_b), c_a ascending), frame
 * as 3 planes (u_x, u_y, T), and the 2-vector reference velocity the FP32
 * moments are taken about (nullable).  Synchronises the stream. */
POND_API pond_status pond_export_state(pond_ctx *c, double *f, double *g, double *frame, double *u_ref);

/* Load a raw state in the layout of pond_export_state (FP32 contexts round to
 * float).  u_ref may be NULL (mass-weighted mean velocity).  Resets the
 * counters.  Synchronises the stream. */
POND_API pond_status pond_import_state(pond_ctx *c, const double *f, const double *g, const double *frame,
                              const double *u_ref);

/* Launch configuration of the step kernel (performance only: every
 * configuration computes the same numbers, bit for bit).
 *   kernel:    POND_KERNEL_TILED (default) stages each block's source region in
 *              LDS; POND_KERNEL_GLOBAL reads every tap from HBM (reference).
 *   tile:      POND_TILE_* block shape of the tiled kernel (destination nodes).
 *   lds_nodes: LDS capacity per block, in nodes (20 moments each: 80 B in FP32,
 *              160 B in FP64); taps outside the staged region read HBM.
 * pond_set_tuning validates the values (POND_ERR_INVALID_ARG otherwise);
 * lds_nodes <= 0 selects the default for the tile. */
enum { POND_KERNEL_TILED = 0, POND_KERNEL_GLOBAL = 1 };
enum { POND_TILE_16x16 = 0, POND_TILE_32x8 = 1, POND_TILE_16x8 = 2, POND_TILE_8x8 = 3,
       POND_TILE_256x1 = 4, POND_TILE_64x1 = 5 };
typedef struct {
    int32_t kernel;
    int32_t tile;
    int32_t lds_nodes;
    int32_t reserved;
} pond_tuning;

POND_API pond_status pond_get_tuning(pond_ctx *c, pond_tuning *out);
POND_API pond_status pond_set_tuning(pond_ctx *c, const pond_tuning *t);

/* Kernel timing on the context stream, for measurement.  While enabled,
 * pond_step brackets each of its launches with HIP events; the results give
 * the summed device time of the moment pre-pass and of the step kernel over
 * the launches since profiling was enabled. */
typedef struct {
    int64_t launches;       /* steps timed */
    double prepass_ms;      /* summed duration of the moment pre-pass launches */
    double step_ms;         /* summed duration of the step-kernel launches */
} pond_profile_t;

/* enable != 0 starts (and clears) timing; 0 stops it and drops pending events. */
POND_API pond_status pond_profile_enable(pond_ctx *c, int enable);

/* Synchronise, then report the timing accumulated since pond_profile_enable(c, 1). */
POND_API pond_status pond_profile_read(pond_ctx *c, pond_profile_t *out);

/* Release the context and the memory it allocated.  NULL-safe. */
POND_API pond_status pond_destroy(pond_ctx *c);

/* Static description of a status code (never NULL). */
POND_API const char *pond_status_string(pond_status s);

/* Message of the last error on the calling thread ("" if none). */
POND_API const char *pond_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* POND_H */
