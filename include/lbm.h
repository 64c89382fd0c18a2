/*
 * lbm.h - C ABI of the MI355X library for the phase-field lattice Boltzmann
 * method for insoluble surfactant transport in two-phase flows
 * (Zhan, Liang, Chai, Shi, arXiv:2408.15654).
 *
 * One simulation ("handle") advances three coupled D2Q9 lattice Boltzmann
 * fields on one GPU:
 *   f  conservative Allen-Cahn phase field phi       Sec. 3.1, Eqs. (21)-(24)
 *   g  interface-confined surfactant psi             Sec. 3.2, Eqs. (25)-(28)
 *   h  consistent Navier-Stokes (u, P)               Sec. 3.3, Eqs. (29)-(33)
 * with the capillary and Marangoni force of Eq. (18), the mass flux of
 * Eq. (16) and the equations of state (19)/(20).  All lattice quantities are
 * in lattice units (dx = dt = 1, c_s^2 = 1/3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout   Host fields are float64 arrays of nx*ny values, row-major with x
 *          fastest: site (x, y) is element y*nx + x.
 * Memory   The caller owns the device workspace (size from
 *          lbm_workspace_bytes) and must keep it alive until lbm_destroy.
 *          Host arrays are only read or written during the call.
 * Streams  All device work is enqueued on the HIP stream given to
 *          lbm_create (NULL = the null stream).  lbm_step does not wait for
 *          the device; lbm_read_fields, lbm_moments and lbm_get_state
 *          synchronise the stream.
 * Errors   Every call returns an lbm_status; no C++ exception crosses the
 *          ABI.  A call that fails before it changes device state leaves
 *          the simulation as it was; one that fails after (a HIP error
 *          while lbm_init_fields or lbm_set_state overwrite the state, or
 *          a launch failure after lbm_step has enqueued some steps) leaves
 *          no valid state, and lbm_step returns LBM_ESTATE until
 *          lbm_init_fields or lbm_set_state succeed.  lbm_last_error gives
 *          a message.  A non-finite value produced on
 *          the device raises a sticky device flag that the next
 *          synchronising call reports as LBM_ENONFINITE; after that,
 *          lbm_step returns LBM_ESTATE until lbm_init_fields or
 *          lbm_set_state.
 * Threads  A handle is not thread-safe; distinct handles are independent.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* invalid argument or parameter */
  LBM_ENOMEM = -2,     /* workspace too small */
  LBM_EDEVICE = -3,    /* HIP runtime error */
  LBM_ENONFINITE = -4, /* the device produced a NaN or Inf (or, with
                          LBM_FP16DEV, a scaled deviation beyond the float16
                          range, which would be stored saturated) */
  LBM_ESTATE = -5      /* no valid state (not initialised, or after ENONFINITE) */
} lbm_status;

/* Storage precision of the populations.  LBM_FP64: float64 storage and
 * arithmetic.  LBM_FP32: float32 storage and arithmetic.  LBM_FP16DEV: each
 * population stored as a float16 deviation, scaled by a power of two, with
 * float32 arithmetic and float32 phi, psi: f_i - w_i phi and g_i - w_i psi
 * (the rest equilibria of Eqs. (22), (26)), and h_i - 3 w_i (P + c_i . rho u)
 * (the part of Eq. (30) linear in P and rho u), each relative to the stored
 * values of the site that wrote it.  The float16 values are rounded
 * stochastically (reproducibly: the random bits are a hash of the values
 * and the site), and a site's rounding errors of f_1..f_8, g_1..g_8 are
 * carried into f_0, g_0, so the sums of phi and psi change by one rounding
 * per site and step. */
typedef enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16DEV = 2 } lbm_precision;

/* Equation of state sigma(psi): linear Eq. (20) or Langmuir Eq. (19). */
typedef enum { LBM_EOS_LINEAR = 0, LBM_EOS_LANGMUIR = 1 } lbm_eos;

/* Where the velocity comes from.  LBM_FLOW_NS: the Navier-Stokes LB of
 * Sec. 3.3, coupled to phi and psi.  LBM_FLOW_PRESCRIBED: the velocity is
 * the field given to lbm_init_fields, held fixed, as in the drop-convection
 * test of Sec. 4.2; only the phase-field and surfactant LBs evolve (f, g),
 * the time differences of Eqs. (22), (26) become (phi - phi_prev) u and
 * (psi - psi_prev) u, and lbm_read_fields returns that u and P = 0. */
typedef enum { LBM_FLOW_NS = 0, LBM_FLOW_PRESCRIBED = 1 } lbm_flow;

/* Problem parameters, named after the paper's statement of the problem.
 * Relaxation rates follow from the transport coefficients:
 *   1/s1^f = M/c_s^2 + 1/2        (Eq. (23), tau_phi = 3M + 1/2)
 *   1/s1^g = D/c_s^2 + 1/2        (Eq. (28), tau_psi = 3D + 1/2)
 *   1/s2^h = mu/(rho c_s^2) + 1/2 (Eq. (33), per site, tau_f = 3 mu/rho + 1/2)
 * The remaining rates of S^k (Eq. (34)) are free and taken from s_free. */
typedef struct {
  int32_t nx, ny;       /* lattice sites; nx, ny >= 3; x is periodic; one
                           copy of the 26 population planes must stay within
                           0xFFFFFF00 bytes (26 nx ny x 8, 4 or 2 bytes by
                           precision: squares up to 4544^2, 6426^2, 9088^2) */
  int32_t walls_y;      /* 0: periodic in y; 1: half-way bounce-back walls
                           below row 0 and above row ny-1 (Sec. 4)          */
  int32_t eos;          /* lbm_eos                                          */
  int32_t precision;    /* lbm_precision                                    */
  int32_t flow;         /* lbm_flow                                         */
  double u_wall_bot;    /* tangential (x) speed of the bottom wall          */
  double u_wall_top;    /* tangential (x) speed of the top wall             */
  double phiA, phiB;    /* order parameter in fluids A and B, phiA > phiB   */
  double W;             /* interface width, > 0                             */
  double M;             /* mobility M_phi, > 0                              */
  double D;             /* surfactant diffusivity, > 0                      */
  double r;             /* normal-diffusion ratio of Eq. (3), >= 0 (1 is the
                           paper's LB model, Eq. (26))                      */
  double rhoA, rhoB;    /* densities, > 0 (Eq. (15))                        */
  double muA, muB;      /* dynamic viscosities, > 0 (Eq. (15))              */
  double sigma0;        /* clean-interface surface tension, >= 0            */
  double beta;          /* elasticity number E_0 of Eqs. (19)-(20)          */
  double gx, gy;        /* body force per unit mass: F_b = rho (gx, gy)     */
  double s_free[3][3];  /* free rates: [0] f: s2,s3,s4  [1] g: s2,s3,s4
                           [2] h: s1,s3,s4; each in (0, 2)                  */
  double fp16_scale[3]; /* LBM_FP16DEV only: power-of-two scale of the
                           stored deviations of f, g, h (0 = default)       */
} lbm_params;

/* Domain-wide sums of the current time level, accumulated in float64. */
typedef struct {
  int64_t step;      /* time steps taken since lbm_init_fields           */
  double sum_phi;    /* sum of phi                                       */
  double sum_psi;    /* sum of psi (total surfactant)                    */
  double mom_x;      /* sum of rho ux                                    */
  double mom_y;      /* sum of rho uy                                    */
  double kinetic;    /* sum of rho |u|^2 / 2                             */
  double max_u;      /* max |u|                                          */
  int32_t nonfinite; /* 1 if any of phi, psi, u is not finite            */
  int32_t pad;
} lbm_moments_t;

typedef struct lbm_handle lbm_handle;

/* Bytes of device workspace a simulation with these parameters needs
 * (populations twice, per-site history, float64 scratch for read-back).
 * Returns 0 if the parameters are invalid. */
size_t lbm_workspace_bytes(const lbm_params *params);

/* Validate params and carve the caller's device workspace.
 * dev_ws: device pointer, 256-byte aligned, ws_bytes >= lbm_workspace_bytes.
 * hip_stream: a hipStream_t (or NULL).  *out receives the handle.
 * Errors: LBM_EINVAL (bad parameter, see the struct), LBM_ENOMEM (workspace
 * too small), LBM_EDEVICE. */
lbm_status lbm_create(const lbm_params *params, void *dev_ws, size_t ws_bytes,
                      void *hip_stream, lbm_handle **out);

/* Set the initial state from host float64 fields (nx*ny each): phi, psi,
 * ux, uy.  Post-collision populations become the equilibria of Eqs. (22),
 * (26), (30) with P = 0 and S from Eq. (16); the stored previous time level
 * is these fields, so the first time differences are taken against them.
 * Computed in float64 on the device, then rounded to the storage precision.
 * Resets the step counter and the non-finite flag.
 * Errors: LBM_EINVAL (NULL array, non-finite value, psi >= 1 with the
 * Langmuir EOS), LBM_EDEVICE. */
lbm_status lbm_init_fields(lbm_handle *h, const double *phi, const double *psi,
                           const double *ux, const double *uy);

/* Advance nsteps >= 0 time steps: each is one launch of the fused
 * stream-collide kernel (pull streaming with half-way bounce-back, the
 * gradient stencils, forces, closures (32a)-(32b), and the three MRT
 * collisions of Eqs. (21), (25), (29) in moment space).  Asynchronous.
 * Errors: LBM_EINVAL (nsteps < 0), LBM_ESTATE, LBM_EDEVICE. */
lbm_status lbm_step(lbm_handle *h, int64_t nsteps);

/* Macroscopic fields of the current time level (phi, psi by Eqs. (24),
 * (27); u and P by Eqs. (32a)-(32b)) into host float64 arrays of nx*ny
 * values.  A NULL pointer skips that field.  Synchronises the stream.
 * Errors: LBM_ESTATE, LBM_ENONFINITE, LBM_EDEVICE. */
lbm_status lbm_read_fields(lbm_handle *h, double *phi, double *psi, double *ux,
                           double *uy, double *P);

/* Float64 domain sums of the current time level (deterministic order):
 * the conserved totals of the phase field (sum of phi, Eq. (24)) and of
 * the surfactant (sum of psi, Eq. (27)), the momentum and kinetic energy of
 * the velocity of Eq. (32a) with rho(phi) of Eq. (15), and max |u|.
 * Synchronises the stream.  Errors: LBM_EINVAL (NULL out), LBM_ESTATE,
 * LBM_ENONFINITE, LBM_EDEVICE. */
lbm_status lbm_moments(lbm_handle *h, lbm_moments_t *out);

/* For callers that cannot allocate device memory or wait for the device:
 * code under HIP graph capture and tight serving loops.  The float64 sums
 * of lbm_moments, enqueued on the handle's stream and written to device
 * memory, with no allocation, no host transfer and no synchronisation:
 *   dev_out[0..6] = sum phi, sum psi, mom_x, mom_y, kinetic, max |u|,
 *                   non-finite (1.0 if phi, psi or u is not finite, else 0.0)
 * in the order and with the values lbm_moments gives (the same kernels).
 * dev_out: device memory on the handle's device for 7 doubles, owned by
 * the caller; it holds the results once the stream reaches this point.
 * The read-back planes and partial sums live in a static buffer the
 * library holds on each device (32.1 MiB, for grids of up to 524288 =
 * 2^19 sites), not in the handle's workspace; every call on one device
 * shares it, so calls that may overlap on one device (different streams,
 * different threads) race and must be ordered by the caller.  Nothing in
 * it needs clearing: each call writes all it reads.  The sticky
 * non-finite flag of the step is not read (that would synchronise); use
 * dev_out[6], or the next synchronising call.
 * Errors: LBM_EINVAL (NULL dev_out, more than 524288 sites), LBM_ESTATE
 * (no valid state), LBM_EDEVICE (launch failure, or no address of the
 * static buffer on this device). */
lbm_status lbm_moments_async(lbm_handle *h, double *dev_out);

/* Shape of fluid A at the current time level, float64, from the phase
 * field phi (c = (phi - phi_B)/(phi_A - phi_B) is the fluid-A fraction):
 * the quantities the paper follows for a sheared drop (interface length,
 * Sec. 4.4) and the Taylor deformation.  For a domain holding one drop
 * they describe that drop; with several drops, area and length are totals
 * and the moments are those of all fluid A together. */
typedef struct {
  double area;          /* sum of c                                          */
  double cx, cy;        /* centroid: circular mean along periodic directions,
                           plain mean between walls (site units)             */
  double Ixx, Ixy, Iyy; /* second moments of c about the centroid, / area,
                           minimum-image displacements                       */
  double length;        /* interface length: sum |grad phi| / (phi_A - phi_B),
                           isotropic D2Q9 gradient                           */
  double taylor_D;      /* (L - B)/(L + B), L, B = 2 sqrt(eigenvalues of I)  */
  double angle;         /* major axis from +x, radians, in (-pi/2, pi/2]     */
} lbm_shape_t;

/* Shape diagnostics of the current level, reduced on the device in float64
 * in a fixed order (synchronising).  EINVAL: out NULL or no fluid A;
 * ESTATE / ENONFINITE as lbm_moments. */
lbm_status lbm_shape(lbm_handle *h, lbm_shape_t *out);

/* Checkpoint: the raw state (populations, previous level, step counter) in
 * storage precision.  lbm_state_bytes gives the size; lbm_get_state copies
 * it to host memory (synchronising), lbm_set_state restores it, after which
 * stepping continues bit for bit as from the saved point.
 * Errors: LBM_EINVAL (NULL or size mismatch), LBM_ENONFINITE (get),
 * LBM_ESTATE (get before init), LBM_EDEVICE. */
size_t lbm_state_bytes(const lbm_handle *h);
lbm_status lbm_get_state(lbm_handle *h, void *host_buf, size_t bytes);
lbm_status lbm_set_state(lbm_handle *h, const void *host_buf, size_t bytes);

/* Release the handle (not the caller's workspace), after waiting for the
 * work it enqueued on its stream, so the workspace may be freed or reused
 * as soon as this returns.  NULL is ignored. */
void lbm_destroy(lbm_handle *h);

/* Message of the last failed call on h (or of the last failed lbm_create
 * when h is NULL).  Valid until the next call on h. */
const char *lbm_last_error(const lbm_handle *h);

/* Rows of lattice each wavefront of the step kernel walks through (its tile
 * height).  The rows are cut into one band per XCD (the hardware deals
 * workgroups to the 8 XCDs round-robin); each band is walked in tiles of
 * this height and ends in a few 1-row tiles, so the launch drains quickly.
 * 0 restores the default plan: for a grid too small to fill the device, the
 * shortest tiles whose wavefronts all fit on it at once (a step then takes
 * about one wavefront's walk down its tile); for float16 storage with two
 * columns per lane, one tile per wavefront slot of the device when such
 * tiles are at most 24 rows high; otherwise a height tuned for large grids.
 * Results do not depend on the tiling.
 * Errors: LBM_EINVAL (< 0 or > 4096). */
lbm_status lbm_set_tile_rows(lbm_handle *h, int32_t rows);

/* The single-grid tile plan in use: plan[0] the tile height, plan[1] the
 * rows at the end of each XCD's band walked in short tiles, plan[2] the
 * height of those (the last may be lower).  plan is host memory of 3
 * int32_t, written only on success.  Errors: LBM_EINVAL (NULL). */
lbm_status lbm_get_tile_plan(const lbm_handle *h, int32_t *plan);

/* The step kernel variant lbm_step launches for this handle, named as a
 * profiler prints its template arguments, e.g.
 * "lbm_step_kernel<F32, 2, false, true, true>": storage (F64, F32, F16; F64C
 * and F32C store with the default cache policy), columns per lane, r != 1,
 * rho_A != rho_B, Navier-Stokes velocity.  Valid while the handle lives;
 * "lbm_step_kernel" for a NULL handle. */
const char *lbm_step_kernel_name(const lbm_handle *h);

/* ----------------------------------------------------------------------
 * Batches: many independent simulations advanced together.
 *
 * A batch owns no memory of its own on the device: the caller gives one
 * workspace (its HBM budget), from which the batch carves its metadata and,
 * for every admitted simulation, the same workspace a single handle would
 * use.  Simulations may differ in size, parameters and precision.  Every
 * lbm_batch_step advances all admitted simulations that still have steps
 * left, in launches of one persistent kernel per kernel variant present
 * (storage precision; one or two columns per lane, two for float32 and
 * float16 storage with even nx; Navier-Stokes or prescribed flow; r == 1
 * or not; equal densities or not); a chunk of those launches is captured
 * once as a HIP graph and replayed.  The
 * arithmetic of each simulation is exactly that of lbm_step on its own
 * (bitwise), whatever the batch holds and whatever the schedule.
 *
 * Simulations join with lbm_batch_submit while others run (admitted as
 * workspace and ids allow) and leave with lbm_batch_retire, so a request
 * loop can keep the device busy with a changing set of solves.
 * All calls are made from one host thread; work goes to the stream given
 * to lbm_batch_create.  Status codes as above; lbm_batch_last_error gives
 * the message of the last failure.
 * ---------------------------------------------------------------------- */
typedef struct lbm_batch lbm_batch;

/* How a batch maps tiles to wavefronts.  rows: tile height for every
 * simulation (0 = each simulation's default).  grid_waves: wavefronts per
 * launch of each variant's persistent kernel (0 = one wavefront per tile).
 * chunk: steps per captured graph, 1..1024. */
typedef struct {
  int32_t rows;
  int32_t grid_waves;
  int32_t chunk;
  int32_t reserved; /* must be 0 */
} lbm_schedule;

/* Device bytes one simulation with these parameters takes from a batch
 * workspace (0 if the parameters are invalid). */
size_t lbm_batch_instance_bytes(const lbm_params *params);

/* Bytes of batch metadata for up to max_instances simulations; the
 * workspace must hold this plus the simulations' own bytes. */
size_t lbm_batch_overhead_bytes(int32_t max_instances);

/* Create a batch over dev_ws (256-byte aligned, ws_bytes long, owned by the
 * caller and kept alive until lbm_batch_destroy) for at most max_instances
 * simultaneous simulations (1..65536).  Default schedule: rows 0,
 * grid_waves 0, chunk 32.  EINVAL: bad arguments; ENOMEM: the workspace
 * cannot hold the metadata; EDEVICE: HIP failure. */
lbm_status lbm_batch_create(int32_t max_instances, void *dev_ws, size_t ws_bytes,
                            void *hip_stream, lbm_batch **out);

/* Admit one simulation: validate params as lbm_create does, take
 * lbm_batch_instance_bytes(params) from the workspace, set the initial
 * state from host float64 fields as lbm_init_fields does, and give it
 * nsteps steps to run.  The copy and initialisation run on a stream of the
 * batch's own, so simulations enqueued earlier on the caller's stream keep
 * stepping meanwhile; the call returns once the new state is in place
 * (it waits for that stream only) and the simulation joins the next
 * lbm_batch_step.  *id receives its id (>= 0).  ENOMEM: no free id or not
 * enough contiguous free workspace now (nothing is changed; retry after a
 * retire).  EINVAL: bad parameters or fields. */
lbm_status lbm_batch_submit(lbm_batch *b, const lbm_params *params, const double *phi,
                            const double *psi, const double *ux, const double *uy,
                            int64_t nsteps, int32_t *id);

/* Advance every admitted simulation by min(nsteps, its remaining steps);
 * asynchronous.  EINVAL: nsteps < 0.  A simulation whose state went
 * non-finite keeps stepping until a synchronising call on it reports it. */
lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps);

/* Steps simulation id still has to run (0 = finished).  No device work. */
lbm_status lbm_batch_remaining(const lbm_batch *b, int32_t id, int64_t *remaining);

/* As lbm_read_fields / lbm_moments for simulation id (synchronising). */
lbm_status lbm_batch_read_fields(lbm_batch *b, int32_t id, double *phi, double *psi,
                                 double *ux, double *uy, double *P);
lbm_status lbm_batch_moments(lbm_batch *b, int32_t id, lbm_moments_t *out);

/* As lbm_shape for simulation id (synchronising). */
lbm_status lbm_batch_shape(lbm_batch *b, int32_t id, lbm_shape_t *out);

/* Remove simulation id and return its workspace (synchronising). */
lbm_status lbm_batch_retire(lbm_batch *b, int32_t id);

/* Largest workspace block a simulation could be admitted into now. */
size_t lbm_batch_free_bytes(const lbm_batch *b);

/* Replace the schedule (EINVAL if out of range).  Results do not change. */
lbm_status lbm_batch_set_schedule(lbm_batch *b, const lbm_schedule *s);
lbm_status lbm_batch_get_schedule(const lbm_batch *b, lbm_schedule *s);

/* Autotuner: time probe_steps steps of the current batch under each
 * candidate schedule (tile heights 4, 8, 16 and each simulation's default;
 * one wavefront per tile or 4, 8, 16 persistent wavefronts per compute
 * unit) and keep the fastest per site update; *chosen (may be NULL)
 * receives it.  The probe steps are real steps of the simulations (their
 * remaining counts go down); results are the same under every schedule.
 * Synchronising. */
lbm_status lbm_batch_autotune(lbm_batch *b, int64_t probe_steps, lbm_schedule *chosen);

/* Synchronise and free the batch (the workspace stays the caller's). */
void lbm_batch_destroy(lbm_batch *b);
const char *lbm_batch_last_error(const lbm_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
