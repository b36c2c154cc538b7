/*
 * lbm.h -- C ABI of the gfx950 (MI355X) implementation of one time step of the
 * three coupled D2Q9 lattice Boltzmann equations of
 *   L. Wang, K. He, H. Wang, "Phase-field-based lattice Boltzmann model for
 *   simulating thermocapillary flows", arXiv:2306.11320:
 *   - the conservative Allen-Cahn LBE for the order parameter phi (Sec. 3.1, Eq. 14),
 *   - the incompressible Navier-Stokes LBE forced by the capillary and Marangoni
 *     stress F_s (Sec. 3.1; force of Eq. 11),
 *   - the modified thermal LBE whose evolution carries the heat-capacitance and
 *     conductivity contrasts (Sec. 3.2, Eq. 28),
 * with isotropic D2Q9 gradient/Laplacian stencils for phi and T.
 *
 * Units are lattice units: dx = dt = 1, c_s^2 = 1/3 (Sec. 4 preamble).
 * phi = -1 marks the light fluid and phi = +1 the heavy fluid (Sec. 2).
 *
 * Conventions shared by every call:
 *   - All calls return int: LBM_OK (0) or a negative LBM_E* code.  No C++
 *     exception crosses the ABI.  lbm_last_error() returns a thread-local text
 *     describing the last failure of the calling thread.
 *   - Host field arrays are row-major with x fastest: element (i, j) is at
 *     index j*nx + i, i in [0, nx), j in [0, ny).  Node (i, j) sits at
 *     x = i, y = j; halfway walls lie at x = -1/2, nx - 1/2, y = -1/2, ny - 1/2.
 *   - Population arrays are [9][ny][nx] in the D2Q9 order c_0 = (0,0),
 *     c_1..4 = (1,0),(0,1),(-1,0),(0,-1), c_5..8 = (1,1),(-1,1),(-1,-1),(1,-1)
 *     (Sec. 4 preamble).
 *   - Device memory and the HIP stream belong to the caller.  A context borrows
 *     them: destroy the context before freeing the workspace.  The library
 *     never allocates or frees device memory; it owns only host objects and the
 *     HIP graphs it captures on the caller's stream.
 *   - Work is enqueued asynchronously on the stream given to lbm_init, except
 *     where a call says it synchronizes.
 *   - A context must not be used from two threads at once.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 2u

/* Collision models (lbm_params.collision). */
enum { LBM_BGK = 0, LBM_TRT = 1 };

/* Forms of the capillary term of the interfacial force (lbm_params.force_form). */
enum { LBM_FORCE_EQ11 = 0, LBM_FORCE_POTENTIAL = 1 };

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* invalid argument or parameter set */
    LBM_ENOSPACE = -2,   /* workspace smaller than lbm_workspace_bytes() */
    LBM_EHIP = -3,       /* a HIP runtime call failed */
    LBM_EUNSTABLE = -4,  /* diagnostics found NaN/Inf or |u| above the limit */
    LBM_ESTATE = -5      /* call not valid in the context's current state */
};

/* Storage precision of the populations. */
enum {
    LBM_FP64 = 0,     /* FP64 storage and arithmetic */
    LBM_FP32_DEV = 1  /* FP32 storage of deviations from the rest equilibrium
                         (phi0_dev, T0_dev, p = 0), FP32 arithmetic; the
                         reductions of lbm_diagnostics stay FP64 */
};

/* Boundary kind of one side. */
enum {
    LBM_BC_PERIODIC = 0,       /* both sides of the axis must be periodic */
    LBM_BC_WALL_T = 1,         /* halfway bounce-back no-slip wall (Sec. 4.1) with a
                                  Dirichlet temperature T_w(s) imposed by
                                  anti-bounce-back */
    LBM_BC_WALL_ADIABATIC = 2, /* halfway bounce-back no-slip wall, zero heat flux */
    LBM_BC_INLET = 3,          /* fully developed inflow 6 u_in s'(H-s')/H^2 along
                                  the inward normal, phi = phi_in, T = T_in (Sec. 4.3) */
    LBM_BC_OUTLET = 4          /* open outflow (Sec. 4.3): anti-bounce-back at
                                  pressure 0 with the node's own u, phi and T */
};

enum { LBM_SIDE_XLO = 0, LBM_SIDE_XHI = 1, LBM_SIDE_YLO = 2, LBM_SIDE_YHI = 3 };

/* Element type of the output buffers of lbm_fields. */
enum { LBM_OUT_F64 = 0, LBM_OUT_F32 = 1 };

/* Problem statement of Sec. 2 and Sec. 4 (two fluids, sigma(T), W, mobility). */
typedef struct lbm_params {
    uint32_t abi_version;  /* must be LBM_ABI_VERSION */
    uint32_t nx, ny;       /* lattice size, each >= 3; one time level of the
                              populations (nx, rounded up to 16 in FP32 unless x
                              is periodic and 64 <= nx <= 256, times ny,
                              rounded up to 64, times 27 values) must stay
                              below 4 GiB */
    uint32_t precision;    /* LBM_FP64 or LBM_FP32_DEV */
    uint32_t bc[4];        /* boundary kind per side: x-lo, x-hi, y-lo, y-hi */
    uint32_t grad_mode;    /* 0: unit normal of the Allen-Cahn source and grad T of
                              the thermal source from the local moments (Sec. 3.1,
                              Sec. 3.2); 1: both from the stencils */
    uint32_t n_bubbles;    /* light-phase regions tracked by lbm_diagnostics (0..4) */
    uint32_t collision;    /* LBM_BGK: the single-relaxation-time collisions of Sec. 3;
                              LBM_TRT: two relaxation times for the NS and thermal LBEs
                              (the extension Sec. 3 names), see trt_magic */
    uint32_t force_form;   /* capillary term of the interfacial force F_s of Eq. 11:
                              LBM_FORCE_EQ11: (sigma/W^2) mu_phi grad phi, the paper's
                              final form; LBM_FORCE_POTENTIAL: -(sigma/W^2) phi grad mu_phi,
                              equal up to a gradient (absorbed by the pressure, which then
                              lacks the jump sigma/W^2 * 3 sqrt2 W/4 * phi mu_phi); mu_phi on
                              the one-node ring takes phi extended to a second ring by the
                              same ghost rules */
    /* fluid properties; _l: light (phi = -1), _h: heavy (phi = +1); each is
       interpolated linearly in phi (Sec. 4 preamble).  mu is the dynamic
       viscosity, lambda the conductivity, rhocp the heat capacitance rho*c_p. */
    double rho_l, rho_h, mu_l, mu_h, lambda_l, lambda_h, rhocp_l, rhocp_h;
    /* sigma(T) = sigma_ref + sigma_T (T - T_ref) + sigma_TT (T - T_ref)^2 / 2:
       the linear law of Sec. 2 and the parabolic law of Eq. 63 */
    double sigma_ref, sigma_T, sigma_TT, T_ref;
    double W;              /* interface width parameter (W = 3 in Sec. 4) */
    double mobility;       /* M_phi = c_s^2 (tau_phi - 1/2) */
    double trt_magic;      /* LBM_TRT: (tau+ - 1/2)(tau- - 1/2); the part that carries the
                              transport coefficient (even for the viscosity, odd for the
                              conductivity) keeps the single-relaxation time; 3/16 makes
                              halfway bounce-back exact for plane Poiseuille flow */
    double Gx, Gy;         /* uniform additional body force G of Eq. 7 */
    /* wall temperature along each side, s the coordinate along the wall:
       T_w(s) = Tw_mean + Tw_amp cos(Tw_k s) + Tw_slope s   (used by LBM_BC_WALL_T) */
    double Tw_mean[4], Tw_amp[4], Tw_k[4], Tw_slope[4];
    double u_in_mean, phi_in, T_in;  /* inlet mean speed, phi and T */
    double phi0_dev, T0_dev;         /* rest state of the deviation storage; with
                                        LBM_FP64 any value is allowed (0 = plain) */
    double bubble_x[4], bubble_y[4]; /* initial centroids of the tracked regions */
} lbm_params;

/* FP64 diagnostics (computed on the GPU in FP64, deterministic order). */
typedef struct lbm_diag {
    int64_t step;          /* time steps taken since lbm_init */
    double mass_phi;       /* sum phi (conserved by Eq. 14 with these BCs) */
    double vol_light;      /* sum (1 - phi)/2, light-phase volume */
    double heat;           /* sum rho c_p T */
    double sum_neg;        /* sum over phi < 0 of phi */
    double u_r;            /* droplet velocity of Sec. 4.2: sum phi u_y / sum phi, phi < 0 */
    double ux_r;           /* the same with u_x */
    double xc, yc;         /* phi-weighted centroid of the phi < 0 nodes */
    double max_u;          /* max |u| */
    int64_t n_nonfinite;   /* nodes with a NaN/Inf macroscopic value */
    int64_t n_neg;         /* number of phi < 0 nodes */
    /* per tracked region (Sec. 4.3): phi < 0 nodes go to the nearest previous
       centroid (ties to the lower index); position and velocity phi-weighted */
    double bub_x[4], bub_y[4], bub_ux[4], bub_uy[4], bub_sum[4];
} lbm_diag;

typedef struct lbm_ctx lbm_ctx;

/* Device workspace, in bytes, that lbm_init needs for one lattice. */
size_t lbm_workspace_bytes(const lbm_params* p);

/*
 * Creates a context for one lattice and sets its populations to equilibrium
 * (Sec. 3: f_i^eq, g_i^eq with p = 0, h_i^eq) for the given initial fields,
 * then sets (phi u) at the previous time level equal to the current one, so
 * the first time derivative of phi u (Sec. 4 preamble) is zero.
 *   p            problem statement; copied.
 *   phi0..T0     host arrays of nx*ny doubles; read during the call only.
 *   d_workspace  device memory of ws_bytes >= lbm_workspace_bytes(p), 256-byte
 *                aligned, owned by the caller, not touched by anyone else while
 *                the context lives.
 *   hip_stream   hipStream_t on which all work is enqueued (NULL = default).
 *   out          receives the context.
 * Synchronizes the stream before returning.
 * Errors: LBM_EINVAL (bad sizes, tau <= 1/2, rhocp <= 0, one periodic side with
 * a non-periodic opposite side, NULL pointers), LBM_ENOSPACE, LBM_EHIP.
 * A heat capacitance below 1 is accepted (LBM_OK), but lbm_last_error() then
 * holds a text starting with "warning:": the destination blend of Eq. 28 is a
 * convex combination of h* and the old h only for rho c_p >= 1.
 */
int lbm_init(const lbm_params* p, const double* phi0, const double* ux0, const double* uy0,
             const double* T0, void* d_workspace, size_t ws_bytes, void* hip_stream, lbm_ctx** out);

/*
 * Advances every lattice of the context by n >= 0 time steps: per step one
 * fused kernel computes the zeroth moments, the stencils, F_s, u, p and the
 * time derivative of phi u, the three BGK collisions (Eq. 14, the NS LBE,
 * Eq. 28) and push streaming with the boundary rules.  Asynchronous.
 * Errors: LBM_EINVAL (n < 0, NULL), LBM_EHIP.
 */
int lbm_step(lbm_ctx* c, int64_t n);

/*
 * Writes the macroscopic fields of the current time level into caller-owned
 * device buffers of nx*ny elements of type out_dtype (LBM_OUT_F64/F32); any
 * pointer may be NULL.  phi = sum f_i, T = sum h_i, u from sum c_i g_i + F/2,
 * p from the pressure moment of Sec. 3.1.  Asynchronous.
 * Errors: LBM_EINVAL, LBM_EHIP.
 */
int lbm_fields(lbm_ctx* c, void* d_phi, void* d_ux, void* d_uy, void* d_T, void* d_p, int out_dtype);

/*
 * FP64 reductions over the current time level (see lbm_diag), copied into
 * *out.  Synchronizes the stream.  Returns LBM_EUNSTABLE (with *out filled) if
 * a NaN/Inf is found or max |u| exceeds 0.5.
 */
int lbm_diagnostics(lbm_ctx* c, lbm_diag* out);

/* Modes of lbm_reinit_fields. */
enum { LBM_REINIT_EQUILIBRIUM = 0, LBM_REINIT_SHIFT = 1 };

/*
 * Re-initialises lattice `instance` from caller-owned device fields (nx*ny
 * elements each, x fastest, FP64 if in_dtype is LBM_OUT_F64, FP32 if
 * LBM_OUT_F32) of phi, u, T and the pressure p (d_p may be NULL).
 *   LBM_REINIT_EQUILIBRIUM: populations := the equilibria f^eq and g^eq of
 *     Sec. 3.1 and h^eq of Sec. 3.2 at the given fields (p = 0 if d_p is NULL);
 *   LBM_REINIT_SHIFT: populations += eq(given fields) - eq(current fields of
 *     the lattice), so their non-equilibrium part is kept (the current p is
 *     kept if d_p is NULL).
 * In both modes (phi u) of the previous level is set to the current one, so
 * the first time derivative of (phi u) after the restart is zero.  The step
 * counter is kept.  Asynchronous on the lattice's stream; the fields must stay
 * valid until it has run.  Errors: LBM_EINVAL (NULL field, unknown dtype or
 * mode, bad instance), LBM_EHIP.
 */
int lbm_reinit_fields(lbm_ctx* c, int instance, const void* d_phi, const void* d_ux, const void* d_uy,
                      const void* d_T, const void* d_p, int in_dtype, int mode);

/* Destroys the context (synchronizes its stream first).  NULL is accepted. */
int lbm_destroy(lbm_ctx* c);

/* Text of the calling thread's last error ("" if none).  Never NULL. */
const char* lbm_last_error(void);

/* ---- state access: parity tests and checkpoint/resume ---- */

/*
 * Copies the populations of lattice `instance` out as absolute FP64 values
 * (deviation storage converted back): f, g, h each [9][ny][nx], jprev
 * [2][ny][nx] ((phi u) at the previous time level); any pointer may be NULL.
 * Synchronizes the stream.  Errors: LBM_EINVAL, LBM_EHIP.
 */
int lbm_get_state(lbm_ctx* c, int instance, double* f, double* g, double* h, double* jprev, int64_t* step);

/* Replaces the populations of lattice `instance` (same layout as
 * lbm_get_state; a NULL array is left unchanged).  Synchronizes the stream. */
int lbm_set_state(lbm_ctx* c, int instance, const double* f, const double* g, const double* h,
                  const double* jprev, int64_t step);

/* Size of a raw checkpoint: the native populations, jprev, the step counter and
 * a hash of the parameters, so that a resumed run is bitwise identical.  The
 * populations keep the library's storage layout, which its format tag names
 * (a checkpoint of another layout is refused). */
size_t lbm_checkpoint_bytes(const lbm_ctx* c);
/* Writes the checkpoint into host memory.  Synchronizes the stream. */
int lbm_checkpoint_save(lbm_ctx* c, void* host_buf, size_t bytes);
/* Restores a checkpoint written by a context with identical parameters;
 * LBM_EINVAL if the size, the format tag or the parameter hash differ.
 * Synchronizes. */
int lbm_checkpoint_load(lbm_ctx* c, const void* host_buf, size_t bytes);

/* ---- batched lattices (many parameter-sweep instances in one launch) ---- */

/* Workspace for n lattices of possibly different sizes and parameters (all
 * with the same precision) advanced together. */
size_t lbm_workspace_bytes_batch(const lbm_params* p, int n);

/*
 * Creates a context holding n lattices.  params[k] and the host arrays
 * phi0[k]..T0[k] describe lattice k.  Each lattice evolves exactly as it would
 * alone (bitwise: the per-node arithmetic does not depend on the batching).
 * One lbm_step launch per time step covers every lattice with a persistent
 * grid that walks a flattened (lattice, tile) table.
 * Errors as lbm_init; LBM_EINVAL also if the precisions differ.
 */
int lbm_init_batch(int n, const lbm_params* params, const double* const* phi0, const double* const* ux0,
                   const double* const* uy0, const double* const* T0, void* d_workspace, size_t ws_bytes,
                   void* hip_stream, lbm_ctx** out);

int lbm_instances(const lbm_ctx* c);
/* lbm_fields / lbm_diagnostics for lattice `instance` of a batched context. */
int lbm_fields_instance(lbm_ctx* c, int instance, void* d_phi, void* d_ux, void* d_uy, void* d_T,
                        void* d_p, int out_dtype);
int lbm_diagnostics_instance(lbm_ctx* c, int instance, lbm_diag* out);

/* ---- launch configuration (autotuning) ---- */

/* Number of compiled tile shapes and the shape of tile id (TX x TY nodes).
 * The last two ids (tx = 512 or 256, ty = 0) step every lattice that is
 * periodic in x with 64 <= nx <= 256 in runs of tx consecutive nodes in
 * x-fastest order (one workgroup per run, so rows of any width leave no
 * work-item idle) and the other lattices in 128 x 4 or 64 x 4 tiles; contexts
 * holding a lattice with the potential form of the capillary force take those
 * tiles throughout. */
int lbm_tile_count(void);
int lbm_tile_shape(int id, int* tx, int* ty);
/* Selects the tile shape used by subsequent steps; invalidates captured graphs.
 * Tile shapes change only the launch, never the per-node arithmetic.  The
 * default after lbm_init is 64 x 4 (id 0) in FP64; in FP32 it is 64 x 8 (id 3)
 * when the device holds every 64 x 8 tile of the context's lattices at once,
 * else 64 x 4. */
int lbm_set_tile(lbm_ctx* c, int id);
int lbm_get_tile(const lbm_ctx* c);
/* Sets how many steps one captured HIP graph holds (0 = plain launches; the
 * default is 64).  Invalidates captured graphs. */
int lbm_set_graph_steps(lbm_ctx* c, int steps);
/* Sets the number of workgroups of the persistent grid (0 = one workgroup per
 * tile, the default for a single lattice). */
int lbm_set_grid(lbm_ctx* c, int workgroups);

/* Workgroups of the persistent grid in use (0: one per tile; -1: sized at the
 * next step). */
int lbm_get_grid(const lbm_ctx* c);

/*
 * Tile autotuner: times G = steps_per_trial rounded up to even steps, one
 * replay of a captured graph, with every compiled tile shape (the run ids only
 * if some lattice of the context is stepped in runs; and, for a batched
 * context, a persistent grid of one and two resident waves of workgroups and
 * one workgroup per tile) with HIP events on the context's stream, after an
 * untimed replay of the same graph, then keeps the fastest.  Tile shape and
 * grid change only the launch, never the per-node arithmetic, so the trial
 * steps are ordinary steps: the lattices advance by max(G, 8) warm-up steps
 * plus 2 G steps per trial (and one step where the count is odd).
 * Synchronizes.
 * Outputs may be NULL.  Errors: LBM_EINVAL, LBM_EHIP.
 */
int lbm_autotune(lbm_ctx* c, int steps_per_trial, int* best_tile, int* best_grid, float* best_ms_per_step);

/* Algorithmic HBM traffic of one lattice update: 27 populations read and
 * written plus (phi u) of the previous level read and written. */
size_t lbm_bytes_per_update(int precision);

/* Measurement aid, not part of the method: copies `bytes` (a multiple of 16,
 * both pointers 16-byte aligned, caller-owned device memory) with a plain
 * vector-copy kernel on `hip_stream`.  Its HBM counters and duration calibrate
 * the traffic and bandwidth figures reported for the step kernel.
 * Errors: LBM_EINVAL, LBM_EHIP.  Asynchronous. */
int lbm_copy_probe(const void* d_src, void* d_dst, size_t bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
