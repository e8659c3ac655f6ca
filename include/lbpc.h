/*
 * lbpc: coupled enthalpy / flow lattice Boltzmann step for solid-liquid phase
 * change on one MI355X (gfx950).
 *
 * Method: Li & He, "Three-dimensional lattice Boltzmann models for solid-liquid
 * phase change" (arXiv 1703.02652).  One time step does, for every cell:
 *   - h = sum_a g_a and the enthalpy -> (T, f_l) rule, Eq. (2) (Sec. 2.1);
 *   - D3Q7 enthalpy collision, SRT Eq. (5)-(8) or MRT Eq. (21)-(25) with the
 *     relaxation rule of Eq. (47) (Sec. 2.2-2.4);
 *   - D3Q19 MRT flow collision with Boussinesq buoyancy, Eq. (48)-(56)
 *     (Sec. 2.5), restricted to the liquid by a solid-region forcing that makes
 *     u = f_l (sum f e + F_b / 2) / rho;
 *   - streaming of both distributions with halfway bounce-back walls, fixed-
 *     temperature (anti-bounce-back) and adiabatic thermal walls (Sec. 3).
 *
 * Conventions for every entry point:
 *   - Lattice units: delta_x = delta_t = c = 1.
 *   - Device pointers are HIP device addresses on the current device; host
 *     pointers are ordinary host memory.  The library never allocates device
 *     memory: the caller provides the workspace and every output buffer.
 *   - Cell order is x fastest: cell = x + nx * (y + ny * z).  Population
 *     arrays are planes [q][cell].
 *   - Work is enqueued on the HIP stream given at creation, in order.  Calls
 *     that return host data synchronise that stream.
 *   - Return codes: LBPC_OK (0) or a negative LBPC_E* code; the context keeps
 *     a message for lbpc_last_error().  No C++ exception crosses this ABI.
 *   - A context is not thread-safe; calls on one context must be serialised.
 */
#ifndef LBPC_H_
#define LBPC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBPC_OK = 0,
  LBPC_EINVAL = -1,     /* bad argument or configuration */
  LBPC_EHIP = -2,       /* a HIP runtime call failed */
  LBPC_ENOSPACE = -3,   /* workspace smaller than required */
  LBPC_EUNSTABLE = -4   /* a cavity produced a non-finite or out-of-bound state */
};

/* Face order everywhere: x-, x+, y-, y+, z-, z+ (walls half a cell outside the
 * first and last nodes). */
enum {
  LBPC_PERIODIC = 0,    /* both faces of the pair must be periodic */
  LBPC_DIRICHLET = 1,   /* fixed temperature (anti-bounce-back) + no-slip */
  LBPC_ADIABATIC = 2    /* zero heat flux (bounce-back) + no-slip */
};

/* Population storage.  The shifted formats store f_a - w_a rho0 (the deviation
 * from rest), and the 16-bit ones g_a - w_a C_p,ref T_shift for a = 1..6 (the
 * deviation from rest at T_shift, a per-cavity reference temperature); g_0,
 * which carries the latent heat, is FP64 in the FP64 format, an FP32 value
 * plus a 16-bit correction (40 significant bits, 6 bytes) in the FP32 format
 * and FP32 in the 16-bit ones; the enthalpy -> (T, f_l) update is FP64 and
 * collision arithmetic FP32 for every format but FP64. */
enum { LBPC_FP64 = 0, LBPC_FP32 = 1, LBPC_FP16S = 2, LBPC_BF16S = 3 };
enum { LBPC_SRT = 0, LBPC_MRT = 1 };

/* Field mask bits for lbpc_fields; planes are written in this bit order. */
enum {
  LBPC_FIELD_H = 1, LBPC_FIELD_T = 2, LBPC_FIELD_FL = 4, LBPC_FIELD_RHO = 8,
  LBPC_FIELD_U = 16 /* three planes: u_x, u_y, u_z */
};

/* One cavity (plain data, lattice units).
 * thermal: omega_T fixes the D3Q7 weights w_0 = 1 - 3 omega_T, w_a = omega_T / 2
 *   (Eq. (8)); the conductivity lambda gives chi = lambda / (rho0 cp_ref) and
 *   tau_g = chi / omega_T + 1/2, sigma_chi = 1 / tau_g (Eq. (20), (34)); local
 *   lambda and C_p are linear in f_l between the solid and liquid values.
 *   Default MRT rates: sigma_0..3 = sigma_chi, sigma_4..6 = 2 - sigma_chi
 *   (Eq. (47)); a finite sigma_override[k] replaces rate k (NaN keeps it).
 * flow: nu gives s_nu = 1 / (3 nu + 1/2) (Eq. (59)); s_e, s_eps, s_q, s_pi, s_t
 *   are the remaining diagonal entries of Eq. (52); the buoyancy is
 *   F_z = rho0 g_beta (T - T_ref) (Eq. (55)).  flow = 0 runs the enthalpy
 *   distribution alone with u = 0. */
typedef struct lbpc_config {
  int32_t nx, ny, nz;   /* each >= 1; nx*ny*nz below 2^29 cells per cavity */
  int32_t flow;         /* 0: enthalpy only, 1: coupled D3Q19 flow */
  int32_t enth_model;   /* LBPC_SRT or LBPC_MRT */
  int32_t precision;    /* LBPC_FP64 ... LBPC_BF16S; same for every cavity of a batch */
  int32_t face_bc[6];
  double face_T[6];     /* wall temperature of LBPC_DIRICHLET faces */
  double omega_T, cp_s, cp_l, cp_ref, lambda_s, lambda_l, latent, T_m, rho0;
  double nu, s_e, s_eps, s_q, s_pi, s_t, g_beta, T_ref;
  double sigma_override[7];
  double T_shift;       /* 16-bit formats: g_1..6 stored as g_a - (omega_T / 2) cp_ref T_shift */
} lbpc_config;

typedef struct lbpc_ctx lbpc_ctx;

/* Device bytes the caller must provide to lbpc_create for this batch (state
 * double buffer, parameter and tile tables, wall fields, budget partials).
 * Returns 0 for an invalid configuration. */
size_t lbpc_workspace_bytes(const lbpc_config* cfgs, int32_t batch);

/* Validate cfgs[0..batch), lay out the caller-owned workspace and initialise
 * every cavity at rest: f = w rho0 and g = g^eq(h0(T0), T0, u = 0) (Eq. (7)),
 * with h0 = C_p,s T0 for T0 <= T_m and C_p,l T0 + L above (Eq. (2)).
 * dev_T0: nullable FP64 device array of all cavities' cells back to back
 * (NULL: T0 = T_m everywhere).  hip_stream: hipStream_t (NULL = default).
 * The workspace must stay allocated until lbpc_destroy. */
int lbpc_create(const lbpc_config* cfgs, int32_t batch, void* dev_workspace, size_t bytes,
                const double* dev_T0, void* hip_stream, lbpc_ctx** out);

/* Replace the temperature of one fixed-temperature face by a per-node field
 * (FP64 device array, copied; the caller keeps ownership).  The wall enters
 * through the anti-bounce-back rule g_abar(x) = -g*_a(x) + 2 w_a C_p,ref T_w
 * of every link that crosses the face: the isothermal walls of the paper's
 * cavity problems (Sec. 3.2.2, 3.3: hot wall at T_h, cold wall at T_m), here
 * with a temperature per wall node.  Node layout: x faces [nz][ny], y faces
 * [nz][nx], z faces [ny][nx].  Synchronises the stream (the face mean is kept
 * on the host for the Nusselt number of lbpc_budgets).  LBPC_EINVAL for a bad
 * cavity or face, a face that is not LBPC_DIRICHLET, or a null field. */
int lbpc_set_wall_T(lbpc_ctx* ctx, int32_t cavity, int32_t face, const double* dev_Tw);

/* Advance every cavity by nsteps time steps (asynchronous).  One step is
 * Eq. (5) for g and Eq. (50) for f: both collisions (Eq. (6)-(8) or (21)-(25),
 * and (49)-(54)) take the macroscopic fields of the same pre-collision state
 * (h, T, f_l by Eq. (2); rho, u by Eq. (55)-(56)), then both distributions
 * stream with the wall rules above.  Steps run in captured HIP graphs of up
 * to graph_steps steps (lbpc_set_launch; the remainder in a shorter graph),
 * each closed by the FP64 budget reduction.  Returns LBPC_EINVAL for
 * nsteps < 0 and LBPC_EUNSTABLE, without stepping, once a cavity has been
 * flagged. */
int lbpc_step(lbpc_ctx* ctx, int64_t nsteps);

/* Macroscopic fields of the current (pre-collision) state of one cavity, FP64
 * planes of nx*ny*nz values in mask-bit order into caller-owned dev_out:
 * h = sum_a g_a (Eq. (2)), T and f_l by the enthalpy rule of Eq. (2),
 * rho = sum f (Eq. (56)) and the forced velocity u = f_l (sum f e + F_b / 2)
 * / rho with F_b of Eq. (55) (zero without flow).  Asynchronous.
 * LBPC_EINVAL for a bad cavity, mask 0 or above 31, or a null output. */
int lbpc_fields(lbpc_ctx* ctx, int32_t cavity, uint32_t mask, double* dev_out);

/* Per cavity, 7 FP64 values into host_out[7 * cavity + k]: H = sum h,
 * mass = sum rho, sum f_l (current state), the enthalpy that entered through
 * fixed-temperature walls since creation, the number of steps taken, the
 * enthalpy q that the next step lets in through the x- face if it has a
 * fixed temperature (exact lattice flux of the anti-bounce-back links), and
 * the mean Nusselt number of that face, Eq. (65) (Sec. 3.2.2, 3.3):
 * Nu = q nx / (ny nz chi_l C_p,ref dT), the lattice heat flux per wall node
 * over the conductive flux chi_l C_p,ref dT / nx across the cavity, with
 * chi_l = lambda_l / (rho0 C_p,ref) and dT = (mean wall temperature of the
 * face) - T_m; NaN when the x- face is not fixed-temperature or dT = 0.
 * Deterministic summation order.  Synchronises the stream. */
int lbpc_budgets(lbpc_ctx* ctx, double* host_out);

/* lbpc_budgets for callers that cannot allocate device memory during the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same values into host_out[7 * cavity + k], the same
 * kernels and summation order (so the same bits), with the per-wavefront
 * records and chunk sums of its reductions in a static device array of
 * 16 MiB that the library holds per device until the process ends, instead of
 * the workspace.  It calls no allocating routine (host records go through
 * fixed stack buffers).  The array is shared by every call on a device and
 * keeps the last call's contents (nothing in it needs to start at zero);
 * calls that overlap on one device, from contexts on different streams or
 * threads, race on it.  LBPC_ENOSPACE when the batch needs more scratch than
 * that (about 5 x 8 bytes per 64 cells: up to some 26 million cells), with
 * the size in lbpc_last_error.  Synchronises the stream. */
int lbpc_budgets_noalloc(lbpc_ctx* ctx, double* host_out);

/* Per-cavity status bits (1 = non-finite or out-of-bound state seen; such a
 * cavity is frozen).  Synchronises the stream. */
int lbpc_status(lbpc_ctx* ctx, int32_t* host_flags);

/* Pre-collision populations of one cavity decoded to FP64: dev_f 19 planes
 * (ignored without flow, may be NULL), dev_g 7 planes.  Velocity order of
 * Eq. (48) and Eq. (3). */
int lbpc_get_state(lbpc_ctx* ctx, int32_t cavity, double* dev_f, double* dev_g);
/* Overwrite the state of one cavity from FP64 planes (encoded to the storage
 * format; dev_f ignored without flow). */
int lbpc_set_state(lbpc_ctx* ctx, int32_t cavity, const double* dev_f, const double* dev_g);

/* Raw checkpoint of the whole batch (populations in storage format, budgets
 * and step counter).  lbpc_load of a buffer from lbpc_save restores the run
 * bit for bit.  Synchronise the stream. */
size_t lbpc_state_bytes(const lbpc_ctx* ctx);
int lbpc_save(lbpc_ctx* ctx, void* host_buf, size_t bytes);
int lbpc_load(lbpc_ctx* ctx, const void* host_buf, size_t bytes);

/* Launch configuration.  block: threads (and cells) per tile, 64, 128, 192
 * or 256; grid_blocks: 0 for one workgroup per tile, else a persistent
 * grid (rounded up to a multiple of 8) that strides over the tile queue;
 * graph_steps: steps per captured HIP graph (at most 16, 0 disables
 * graphs); xcd_run: 0..2^24, the queue order.  The MI355X dispatcher sends
 * workgroup b to XCD b mod 8; for xcd_run >= 1 the queue is ordered so that
 * each XCD walks runs of xcd_run consecutive tiles (in the natural order of
 * the cells), the runs of the eight XCDs side by side.  1 is the natural
 * order; a run longer than an eighth of the queue is cut to that length (one
 * contiguous run per XCD).  xcd_run = 0: XCD k takes the tiles whose first row
 * lies in the k-th eighth of the y range, slab after slab.
 * Consecutive steps walk each XCD's share of the queue in opposite
 * directions, so that an XCD first reads what it wrote last in the step before
 * (still in its L2 and in the Infinity Cache).
 * Results do not depend on any of these settings: the state bit for bit, and
 * the budgets for a given block size. */
int lbpc_set_launch(lbpc_ctx* ctx, int32_t block, int32_t grid_blocks, int32_t graph_steps,
                    int32_t xcd_run);
int lbpc_get_launch(const lbpc_ctx* ctx, int32_t* block, int32_t* grid_blocks,
                    int32_t* graph_steps, int32_t* xcd_run);

/* Time every candidate launch configuration (tile size 64/128/256, one
 * workgroup per tile or a persistent grid of 4 workgroups per compute unit,
 * y-blocks per XCD, XCD runs of 1, 2, 4, 8, 16, 32 tiles or one run per XCD)
 * with trial_steps real alternating steps from the current state
 * (without budget partials), re-time the three fastest four times more,
 * interleaved, and keep the fastest of those.  The state is copied to host
 * memory first and restored afterwards, so tuning does not advance the run.
 * host_ms_out (nullable) receives the best average step-kernel time in
 * milliseconds.  Synchronises the stream. */
int lbpc_autotune(lbpc_ctx* ctx, int32_t trial_steps, double* host_ms_out);

/* Time the step kernel as the graphs of lbpc_step run it: a captured graph of
 * 14 back-to-back wall-inflow-partials steps, replayed ceil(nsteps / 14)
 * times between one HIP event pair each on the library's stream; every replay
 * is followed by two untimed eager steps (the second with all partials, which
 * closes the budget ring), so the run advances 16 steps per replay.  The mean
 * time per timed step in milliseconds goes to host_ms_out.  Synchronises. */
int lbpc_time_step_kernel(lbpc_ctx* ctx, int32_t nsteps, double* host_ms_out);

/* Discrete adjoint of the loss L = sum over cells of f_l at the final step
 * (loss = 0) or L / (ny nz), the interface position of a front along x
 * (loss = 1), w.r.t. the wall temperatures and the initial temperature field.
 * Single-cavity contexts in LBPC_FP64 or LBPC_FP32 only.
 *   lbpc_adjoint_workspace_bytes: device bytes for nsteps with a checkpoint every
 *     ckpt_every steps (snapshots, one segment of recomputed states, adjoint
 *     populations).
 *   lbpc_adjoint_forward: run nsteps from the current state, storing
 *     checkpoints in dev_adj_ws; the state is left at the final step; the loss
 *     goes to host_loss (synchronises).  ckpt_every = 1 keeps every state
 *     (nsteps regions: 96^3 x 2000 FP32 steps take 191 GB): each step writes
 *     into its snapshot directly and the reverse sweep recomputes nothing.
 *   lbpc_adjoint_backward: reverse sweep with recomputation per segment (the
 *     forward run leaves the states of its last segment in place, so the first
 *     call recomputes every segment but that one); seed scales the loss
 *     (dL/dL = seed); it may be called again for the same forward run.  dev_dL_dTw: FP64, all six faces'
 *     node fields back to back (layout of lbpc_set_wall_T), zero on faces
 *     that are not fixed-temperature.  dev_dL_dT0: FP64 per cell, the
 *     derivative w.r.t. the initial temperature of lbpc_create (one-sided,
 *     solid side, at T0 = T_m); only valid when the forward started from the
 *     state made by lbpc_create.  Either output may be NULL. */
size_t lbpc_adjoint_workspace_bytes(const lbpc_ctx* ctx, int64_t nsteps, int32_t ckpt_every);
int lbpc_adjoint_forward(lbpc_ctx* ctx, int64_t nsteps, int32_t ckpt_every, int32_t loss,
                         void* dev_adj_ws, size_t bytes, double* host_loss);
int lbpc_adjoint_backward(lbpc_ctx* ctx, double seed, double* dev_dL_dTw, double* dev_dL_dT0);

/* Both passes in one call: lbpc_adjoint_forward(ctx, nsteps, ckpt_every, loss,
 * dev_adj_ws, bytes, host_loss), then lbpc_adjoint_backward with seed 1, so
 * that dev_dL_dTw and dev_dL_dT0 (each nullable) receive dL/dT_w and dL/dT0 of
 * the loss.  The state is left at the final step.  Synchronises. */
int lbpc_adjoint(lbpc_ctx* ctx, int64_t nsteps, int32_t ckpt_every, int32_t loss,
                 void* dev_adj_ws, size_t bytes, double* dev_dL_dTw, double* dev_dL_dT0,
                 double* host_loss);

void lbpc_destroy(lbpc_ctx* ctx);
const char* lbpc_last_error(const lbpc_ctx* ctx);
const char* lbpc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LBPC_H_ */
